// fdtd_tens_adj.hip -- adjoint step of symmetric-tensor media for gfx950.
//
// The forward E update of a tensor domain is E += S M y: y the stretched
// curl of H on every E edge (zero on edges held by a wall), M the node
// assembly (1/8) sum over the eight octants of each node of R^T eps^-1 R
// (Section 2.3).  Its transpose (Section 3.1) runs in three launches per
// step; the last is the split adjoint's H-node pass, shared with the other
// media:
//   k_tadj_ht  per E node: the H-update transpose gathered onto the edge,
//              Ebar^{n+1} -> the new Ebar (no dispersion in tensor media,
//              so the E-update transpose is the identity on E^n);
//   k_tadj_e   per E node: u = S M Ebar (M is symmetric, so it is its own
//              transpose) from the cotangents of the 18 edges and the 15
//              node-tensor entries the node's three edges meet, the E-side
//              absorber memory cotangents, and the node tensor's gradient
//              (the forward curls of the node's six edges from 12 H values
//              away from the absorbing slabs);
//   k_adj_et   u through the transposed absorber recursion and the curl into
//              Hbar (in a Bloch-periodic domain the per-node k_padj_h, whose
//              gathers cross the seams).
// On a periodic axis (Section 2.2) the edges past a seam are those at the
// other end times the real Bloch factor, the node tensors past it repeat.
// k_tadj_ht marches (i, j) columns of kNodeKz planes (fdtd_node_adj.h);
// k_tadj_e takes one node per thread, 64 x-nodes by 4 rows per block, one
// plane per block row of the grid (a z-stride loop beyond the grid's z
// extent).  The passes read set rs of the adjoint state and write set ws,
// like the split adjoint.
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "fdtd_launch.h"
#include "fdtd_node_adj.h"

namespace fdtd {
namespace {

constexpr int kTx = 64, kTy = 4, kMaxGridZ = 65535;

// eps^-1 entry q (xx yy zz xy xz yz) at node (i,j,k), i <= nx, j <= ny: the
// box arrays, the background times the identity outside the box (the
// high-wall nodes included); past a periodic seam (PER: the domain has a
// periodic axis) the node at the other end
template <typename T, bool PER>
__device__ __forceinline__ T tinv_at(const DomDev<T>& d, int q, int i, int j, int k) {
    if constexpr (PER) {
        if (i >= d.n[0] && d.per[0]) i -= d.n[0];
        if (j >= d.n[1] && d.per[1]) j -= d.n[1];
    }
    if (in_box<T>(d.elo, d.ehi, i, j, k)) {
        const long long o =
            ((long long)(k - d.elo[2]) * (d.ehi[1] - d.elo[1]) + (j - d.elo[1])) * d.exs + (i - d.exa);
        return gp(d.tinv[q])[o];
    }
    return q < 3 ? d.epsinv_bg : T(0);
}

// (i, j) one step off the grid in x or y (at most): across a periodic seam
// the node at the other end and the Bloch factor, else false
template <typename T>
__device__ __forceinline__ bool seam_wrap(const DomDev<T>& d, int& i, int& j, T& fac) {
    fac = T(1);
    if (i < 0 || i >= d.n[0]) {
        if (!d.per[0]) return false;
        i += i < 0 ? d.n[0] : -d.n[0];
        fac = d.bsign[0];
    }
    if (j < 0 || j >= d.n[1]) {
        if (!d.per[1]) return false;
        j += j < 0 ? d.n[1] : -d.n[1];
        fac *= d.bsign[1];
    }
    return true;
}

// value of an edge array at the edge starting at (i,j,k); zero off the grid
// past a wall
template <typename T, bool PER>
__device__ __forceinline__ T edge_at(const DomDev<T>& d, const FDTD_GLOBAL T* F, int i, int j, int k) {
    if constexpr (PER) {
        T fac;
        if (k < 0 || k >= d.n[2] || !seam_wrap(d, i, j, fac)) return T(0);
        return fac * F[fidx(d, i, j, k)];
    } else {
        if (i < 0 || j < 0 || k < 0 || i >= d.n[0] || j >= d.n[1] || k >= d.n[2]) return T(0);
        return F[fidx(d, i, j, k)];
    }
}

template <bool PER, typename T>
__device__ __forceinline__ bool emask(const DomDev<T>& d, int c, int i, int j, int k) {
    if constexpr (PER) return e_masked_d(d, c, i, j, k);
    else return e_masked(c, i, j, k);
}

// the forward stretched curl of edge (c, x) from u^n (set fsr), read only;
// zero on an edge a wall holds
template <typename T, bool PER>
__device__ __forceinline__ T fwd_curl(const DomDev<T>& d, int c, const int x[3], int fsr) {
    if constexpr (!PER) {
        if (x[0] < 0 || x[1] < 0 || x[2] < 0 || e_masked(c, x[0], x[1], x[2])) return T(0);
        const long long fo = (long long)fsr * d.fs, f = fidx(d, x[0], x[1], x[2]) + fo;
        const long long st[3] = {1, d.pitch, d.plane};
        const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
        const FDTD_GLOBAL T* H0 = gp(d.H[(c + 2) % 3]);   // differenced along a0
        const FDTD_GLOBAL T* H1 = gp(d.H[(c + 1) % 3]);   // differenced along a1
        const T h0 = H0[f], h0m = x[a0] > 0 ? H0[f - st[a0]] : T(0);
        const T h1 = H1[f], h1m = x[a1] > 0 ? H1[f - st[a1]] : T(0);
        return curl_minus_ro(d, c, x[0], x[1], x[2], h0, h0m, h1, h1m, fsr);
    }
    int w[3] = {x[0], x[1], x[2]};
    T fac;
    if (w[2] < 0 || !seam_wrap(d, w[0], w[1], fac) || e_masked_d(d, c, w[0], w[1], w[2])) return T(0);
    const long long fo = (long long)fsr * d.fs, f = fidx(d, w[0], w[1], w[2]);
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    const FDTD_GLOBAL T* H0 = gp(d.H[(c + 2) % 3]) + fo;   // differenced along a0
    const FDTD_GLOBAL T* H1 = gp(d.H[(c + 1) % 3]) + fo;   // differenced along a1
    int y[3];
    T fb;
    const T h0m = back_node(d, a0, w, y, fb) ? fb * H0[fidx(d, y[0], y[1], y[2])] : T(0);
    const T h1m = back_node(d, a1, w, y, fb) ? fb * H1[fidx(d, y[0], y[1], y[2])] : T(0);
    return fac * curl_minus_ro(d, c, w[0], w[1], w[2], H0[f], h0m, H1[f], h1m, fsr);
}

template <typename T>
__global__ void __launch_bounds__(256) k_tadj_ht(const DomDev<T>* __restrict__ dp, int rs, int ws) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kNodeTx + threadIdx.x % kNodeTx, j = blockIdx.y * kNodeTy + threadIdx.x / kNodeTx;
    const int k0 = blockIdx.z * kNodeKz, k1 = min(k0 + kNodeKz, d.n[2]);
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long wo = (long long)ws * d.as;
    HtGather<T> hg(d, i, j, k0, rs, ws);
    long long f = fidx(d, i, j, k0);
    HtPlane<T> cu = hg.fetch(f), nx;
    for (int k = k0; k < k1; ++k, f += d.plane) {
        if (k + 1 < k1) nx = hg.fetch(f + d.plane);   // plane k+1's loads ahead of plane k's stores
        T et[3];
        hg.gather(k, cu, et);
        gp(d.Ea[0])[f + wo] = et[0];
        gp(d.Ea[1])[f + wo] = et[1];
        gp(d.Ea[2])[f + wo] = et[2];
        cu = nx;
    }
}

// forward field value at (i,j,k) of array F, zero before the first node
template <typename T>
__device__ __forceinline__ T back_val(const DomDev<T>& d, const FDTD_GLOBAL T* F, int i, int j, int k) {
    return (i < 0 || j < 0 || k < 0) ? T(0) : F[fidx(d, i, j, k)];
}

// k_tadj_e's wave target per SIMD.  FP32 at 5 (95 VGPRs, no spills; left
// alone the compiler takes 103 and 4 waves): 5.67 against 6.58 ms at 536^3;
// at 6 (80 VGPRs, 12 spills) 6.24 ms.  FP64 keeps 4 (125 VGPRs; at 5 waves
// it would spill 28).
template <typename T> constexpr int kTadjWaves = sizeof(T) == 8 ? 4 : 5;

template <typename T, bool PER>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kTadjWaves<T>, 8))) k_tadj_e(const DomDev<T>* __restrict__ dp, int rs, int ws, int fsr) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kTx + threadIdx.x % kTx, j = blockIdx.y * kTy + threadIdx.x / kTx;
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long wo = (long long)ws * d.as;
    const FDTD_GLOBAL T* ex = gp(d.Ea[0]) + wo;
    const FDTD_GLOBAL T* ey = gp(d.Ea[1]) + wo;
    const FDTD_GLOBAL T* ez = gp(d.Ea[2]) + wo;
    const T S = d.S, h = T(0.5), q4 = T(0.25);
    for (int k = blockIdx.z; k < d.n[2]; k += gridDim.z) {
        const long long f = fidx(d, i, j, k);
        // Ebar on the edges the three assembled edges of node v = (i,j,k) meet
        // (suffixes: offsets from v; zero off the grid)
        const T x0 = ex[f], x_xm = edge_at<T, PER>(d, ex, i - 1, j, k), x_yp = edge_at<T, PER>(d, ex, i, j + 1, k),
                x_xmyp = edge_at<T, PER>(d, ex, i - 1, j + 1, k), x_zp = edge_at<T, PER>(d, ex, i, j, k + 1),
                x_xmzp = edge_at<T, PER>(d, ex, i - 1, j, k + 1);
        const T y0 = ey[f], y_ym = edge_at<T, PER>(d, ey, i, j - 1, k), y_xp = edge_at<T, PER>(d, ey, i + 1, j, k),
                y_xpym = edge_at<T, PER>(d, ey, i + 1, j - 1, k), y_zp = edge_at<T, PER>(d, ey, i, j, k + 1),
                y_ymzp = edge_at<T, PER>(d, ey, i, j - 1, k + 1);
        const T z0 = ez[f], z_zm = edge_at<T, PER>(d, ez, i, j, k - 1), z_xp = edge_at<T, PER>(d, ez, i + 1, j, k),
                z_xpzm = edge_at<T, PER>(d, ez, i + 1, j, k - 1), z_yp = edge_at<T, PER>(d, ez, i, j + 1, k),
                z_ypzm = edge_at<T, PER>(d, ez, i, j + 1, k - 1);
        // node tensors: v (all six), v+x (xx xy xz), v+y (yy xy yz), v+z (zz xz yz)
        const T a_xx = tinv_at<T, PER>(d, 0, i, j, k), a_yy = tinv_at<T, PER>(d, 1, i, j, k),
                a_zz = tinv_at<T, PER>(d, 2, i, j, k), a_xy = tinv_at<T, PER>(d, 3, i, j, k),
                a_xz = tinv_at<T, PER>(d, 4, i, j, k), a_yz = tinv_at<T, PER>(d, 5, i, j, k);
        const T px_xx = tinv_at<T, PER>(d, 0, i + 1, j, k), px_xy = tinv_at<T, PER>(d, 3, i + 1, j, k),
                px_xz = tinv_at<T, PER>(d, 4, i + 1, j, k);
        const T py_yy = tinv_at<T, PER>(d, 1, i, j + 1, k), py_xy = tinv_at<T, PER>(d, 3, i, j + 1, k),
                py_yz = tinv_at<T, PER>(d, 5, i, j + 1, k);
        const T pz_zz = tinv_at<T, PER>(d, 2, i, j, k + 1), pz_xz = tinv_at<T, PER>(d, 4, i, j, k + 1),
                pz_yz = tinv_at<T, PER>(d, 5, i, j, k + 1);
        const T sx = x0 + x_xm, sy = y0 + y_ym, sz = z0 + z_zm;   // the two edges of each axis at v
        T mx = h * (a_xx + px_xx) * x0;
        mx += q4 * (a_xy * sy + px_xy * (y_xp + y_xpym));
        mx += q4 * (a_xz * sz + px_xz * (z_xp + z_xpzm));
        T my = h * (a_yy + py_yy) * y0;
        my += q4 * (a_xy * sx + py_xy * (x_yp + x_xmyp));
        my += q4 * (a_yz * sz + py_yz * (z_yp + z_ypzm));
        T mz = h * (a_zz + pz_zz) * z0;
        mz += q4 * (a_xz * sx + pz_xz * (x_zp + x_xmzp));
        mz += q4 * (a_yz * sy + pz_yz * (y_zp + y_ymzp));
        T u[3] = {emask<PER>(d, 0, i, j, k) ? T(0) : S * mx, emask<PER>(d, 1, i, j, k) ? T(0) : S * my,
                  emask<PER>(d, 2, i, j, k) ? T(0) : S * mz};
        gp(d.Et[0])[f] = u[0];
        gp(d.Et[1])[f] = u[1];
        gp(d.Et[2])[f] = u[2];
        const bool slab = slab_side(d, 0, i) >= 0 || slab_side(d, 1, j) >= 0 || slab_side(d, 2, k) >= 0;
        // E-side memory cotangents (owner): ybar = +u (term 0), -u (term 1)
        if (slab)
            for (int c = 0; c < 3; ++c) {
                if (emask<PER>(d, c, i, j, k)) continue;
                for (int t = 0; t < 2; ++t)
                    (void)stretch_T(d, d.psiEa, rs, ws, true, (c + 1 + t) % 3, t, 0, i, j, k, t == 0 ? u[c] : -u[c]);
            }
        if (!in_gbox(d, i, j, k)) continue;
        // node gradient.  U, Y: S Ebar and the forward curl on the two edges of
        // each axis b at the node (0: leaving, 1: arriving).  With eps^-1 = A,
        // dJ/dA_ab = 1/8 sum over octants of U_a Y_b; as a symmetric matrix
        // G_aa = 1/2 (U_a0 Y_a0 + U_a1 Y_a1), G_ab = 1/8 (sU_a sY_b + sU_b sY_a)
        // (sums over the two edges); the gradient of eps is Q = -A G A, stored
        // as Q_aa and 2 Q_ab for the entries xx yy zz xy xz yz
        double U[3][2], Y[3][2];
        U[0][0] = (double)(S * x0);
        U[0][1] = (double)(S * x_xm);
        U[1][0] = (double)(S * y0);
        U[1][1] = (double)(S * y_ym);
        U[2][0] = (double)(S * z0);
        U[2][1] = (double)(S * z_zm);
        // stretched curls where the absorber memories of u^n take part, and on
        // a periodic axis's first plane (the back differences cross the seam)
        if (slab || (PER && ((d.per[0] && i == 0) || (d.per[1] && j == 0)))) {
            for (int b = 0; b < 3; ++b)
                for (int s = 0; s < 2; ++s) {
                    int w[3] = {i, j, k};
                    w[b] -= s;
                    Y[b][s] = (double)fwd_curl<T, PER>(d, b, w, fsr);
                }
        } else {      // plain backward-difference curls of the forward H
            const long long fo = (long long)fsr * d.fs;
            const FDTD_GLOBAL T* Hx = gp(d.H[0]) + fo;
            const FDTD_GLOBAL T* Hy = gp(d.H[1]) + fo;
            const FDTD_GLOBAL T* Hz = gp(d.H[2]) + fo;
            const T hx = Hx[f], hx_ym = back_val(d, Hx, i, j - 1, k), hx_zm = back_val(d, Hx, i, j, k - 1),
                    hx_ymzm = back_val(d, Hx, i, j - 1, k - 1);
            const T hy = Hy[f], hy_xm = back_val(d, Hy, i - 1, j, k), hy_zm = back_val(d, Hy, i, j, k - 1),
                    hy_xmzm = back_val(d, Hy, i - 1, j, k - 1);
            const T hz = Hz[f], hz_xm = back_val(d, Hz, i - 1, j, k), hz_ym = back_val(d, Hz, i, j - 1, k),
                    hz_xmym = back_val(d, Hz, i - 1, j - 1, k);
            const bool mx_ = j == 0 || k == 0, my_ = i == 0 || k == 0, mz_ = i == 0 || j == 0;
            Y[0][0] = mx_ ? 0.0 : (double)((hz - hz_ym) - (hy - hy_zm));
            Y[0][1] = (mx_ || i == 0) ? 0.0 : (double)((hz_xm - hz_xmym) - (hy_xm - hy_xmzm));
            Y[1][0] = my_ ? 0.0 : (double)((hx - hx_zm) - (hz - hz_xm));
            Y[1][1] = (my_ || j == 0) ? 0.0 : (double)((hx_ym - hx_ymzm) - (hz_ym - hz_xmym));
            Y[2][0] = mz_ ? 0.0 : (double)((hy - hy_xm) - (hx - hx_ym));
            Y[2][1] = (mz_ || k == 0) ? 0.0 : (double)((hy_zm - hy_xmzm) - (hx_zm - hx_ymzm));
        }
        double G[3][3];
        const double A[3][3] = {{(double)a_xx, (double)a_xy, (double)a_xz},
                                {(double)a_xy, (double)a_yy, (double)a_yz},
                                {(double)a_xz, (double)a_yz, (double)a_zz}};
        for (int a = 0; a < 3; ++a) {
            G[a][a] = 0.5 * (U[a][0] * Y[a][0] + U[a][1] * Y[a][1]);
            for (int b = a + 1; b < 3; ++b) {
                const double g = 0.125 * ((U[a][0] + U[a][1]) * (Y[b][0] + Y[b][1]) +
                                          (U[b][0] + U[b][1]) * (Y[a][0] + Y[a][1]));
                G[a][b] = G[b][a] = g;
            }
        }
        double B[3][3];   // G A
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) B[a][b] = G[a][0] * A[0][b] + G[a][1] * A[1][b] + G[a][2] * A[2][b];
        const long long q = ((long long)(k - d.glo[2]) * (d.ghi[1] - d.glo[1]) + (j - d.glo[1])) *
                                (d.ghi[0] - d.glo[0]) + (i - d.glo[0]);
        static constexpr int qa[6] = {0, 1, 2, 0, 0, 1}, qb[6] = {0, 1, 2, 1, 2, 2};
        for (int p = 0; p < 6; ++p) {
            const int a = qa[p], b = qb[p];
            const double Q = -(A[a][0] * B[0][b] + A[a][1] * B[1][b] + A[a][2] * B[2][b]);
            gp(d.gacc[p])[q] += a == b ? Q : 2.0 * Q;
        }
    }
}

}  // namespace

template <typename T>
void launch_tens_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, bool per, hipStream_t s) {
    const DomDev<T>* dp = (const DomDev<T>*)doms + dom;
    const dim3 gcol((n[0] + kNodeTx - 1) / kNodeTx, (n[1] + kNodeTy - 1) / kNodeTy, (n[2] + kNodeKz - 1) / kNodeKz);
    const dim3 gplane((n[0] + kTx - 1) / kTx, (n[1] + kTy - 1) / kTy, std::min(n[2], kMaxGridZ));
    hipLaunchKernelGGL(k_tadj_ht<T>, gcol, dim3(256), 0, s, dp, rs, ws);
    if (per) hipLaunchKernelGGL((k_tadj_e<T, true>), gplane, dim3(256), 0, s, dp, rs, ws, fsr);
    else hipLaunchKernelGGL((k_tadj_e<T, false>), gplane, dim3(256), 0, s, dp, rs, ws, fsr);
}

template void launch_tens_adj<float>(const void*, int, const int*, int, int, int, bool, hipStream_t);
template void launch_tens_adj<double>(const void*, int, const int*, int, int, int, bool, hipStream_t);

}  // namespace fdtd
