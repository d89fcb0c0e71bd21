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
//              transpose), the E-side absorber memory cotangents, and the
//              node tensor's gradient;
//   k_adj_et   u through the transposed absorber recursion and the curl into
//              Hbar.
// One thread per node, 64 x-nodes by 4 rows per block, one plane per block
// row of the grid (a z-stride loop beyond the grid's z extent).  The passes
// read set rs of the adjoint state and write set ws, like the split adjoint.
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "fdtd_launch.h"

namespace fdtd {
namespace {

constexpr int kTx = 64, kTy = 4, kMaxGridZ = 65535;

// eps^-1 entry q (xx yy zz xy xz yz) at node (i,j,k): the box arrays, the
// background times the identity outside the box (the high-wall nodes included)
template <typename T>
__device__ __forceinline__ T tinv_at(const DomDev<T>& d, int q, int i, int j, int k) {
    if (in_box<T>(d.elo, d.ehi, i, j, k)) {
        const long long o =
            ((long long)(k - d.elo[2]) * (d.ehi[1] - d.elo[1]) + (j - d.elo[1])) * d.exs + (i - d.exa);
        return gp(d.tinv[q])[o];
    }
    return q < 3 ? d.epsinv_bg : T(0);
}

__device__ __forceinline__ int tcomp(int a, int b) {
    return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

// value of an edge array at the edge starting at (i,j,k); zero off the grid
template <typename T>
__device__ __forceinline__ T edge_at(const DomDev<T>& d, const FDTD_GLOBAL T* F, int i, int j, int k) {
    if (i < 0 || j < 0 || k < 0 || i >= d.n[0] || j >= d.n[1] || k >= d.n[2]) return T(0);
    return F[fidx(d, i, j, k)];
}

// (M F)_c at the edge of component c starting at x: at each end node v the
// edge takes eps^-1_cc(v)/2 times its own value and eps^-1_cb(v)/4 times the
// sum over the two b edges meeting at v (leaving and arriving), b != c
template <typename T>
__device__ __forceinline__ T assemble(const DomDev<T>& d, const FDTD_GLOBAL T* const (&F)[3], int c, int i, int j,
                                      int k) {
    const T own = F[c][fidx(d, i, j, k)];
    T acc = T(0);
    for (int end = 0; end < 2; ++end) {
        int v[3] = {i, j, k};
        v[c] += end;
        acc += T(0.5) * tinv_at(d, c, v[0], v[1], v[2]) * own;
        for (int t = 1; t < 3; ++t) {
            const int b = (c + t) % 3;
            int w[3] = {v[0], v[1], v[2]};
            T s = edge_at(d, F[b], w[0], w[1], w[2]);
            w[b] -= 1;
            s += edge_at(d, F[b], w[0], w[1], w[2]);
            acc += T(0.25) * tinv_at(d, tcomp(c, b), v[0], v[1], v[2]) * s;
        }
    }
    return acc;
}

// the forward stretched curl of edge (c, x) from u^n (set fsr), read only;
// zero on an edge a wall holds
template <typename T>
__device__ __forceinline__ T fwd_curl(const DomDev<T>& d, int c, const int x[3], int fsr) {
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

template <typename T>
__global__ void __launch_bounds__(256) k_tadj_ht(const DomDev<T>* __restrict__ dp, int rs, int ws) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kTx + threadIdx.x % kTx, j = blockIdx.y * kTy + threadIdx.x / kTx;
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as;
    const long long st[3] = {1, d.pitch, d.plane};
    for (int k = blockIdx.z; k < d.n[2]; k += gridDim.z) {
        const long long f = fidx(d, i, j, k);
        const int x[3] = {i, j, k};
        for (int e = 0; e < 3; ++e) {
            T acc = T(0);
            if (!e_masked(e, i, j, k)) {
                acc = gp(d.Ea[e])[f + ro];
                // E_e enters H_c's update term t, differenced forward along a:
                // t = 0: c = e+1, a = e+2, sign +; t = 1: c = e+2, a = e+1, sign -.
                // D(p) = E_e(p + a) - E_e(p), so Ebar_e(x) gets Dbar(x - a) - Dbar(x)
                for (int t = 0; t < 2; ++t) {
                    const int c = t == 0 ? (e + 1) % 3 : (e + 2) % 3;
                    const int a = t == 0 ? (e + 2) % 3 : (e + 1) % 3;
                    const T sgn = t == 0 ? T(1) : T(-1);
                    const FDTD_GLOBAL T* hb = gp(d.Ha[c]) + ro;
                    acc -= hT_dbar(d, a, t, sgn, i, j, k, hb[f], rs, ws, false);
                    if (x[a] > 0) {
                        int y[3] = {i, j, k};
                        y[a] -= 1;
                        acc += hT_dbar(d, a, t, sgn, y[0], y[1], y[2], hb[f - st[a]], rs, ws, false);
                    }
                }
            }
            gp(d.Ea[e])[f + wo] = acc;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_tadj_e(const DomDev<T>* __restrict__ dp, int rs, int ws, int fsr) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kTx + threadIdx.x % kTx, j = blockIdx.y * kTy + threadIdx.x / kTx;
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long wo = (long long)ws * d.as;
    const FDTD_GLOBAL T* eb[3] = {gp(d.Ea[0]) + wo, gp(d.Ea[1]) + wo, gp(d.Ea[2]) + wo};
    const T S = d.S;
    for (int k = blockIdx.z; k < d.n[2]; k += gridDim.z) {
        const long long f = fidx(d, i, j, k);
        T u[3];
        for (int c = 0; c < 3; ++c) {
            u[c] = e_masked(c, i, j, k) ? T(0) : S * assemble(d, eb, c, i, j, k);
            gp(d.Et[c])[f] = u[c];
        }
        // E-side memory cotangents (owner): ybar = +u (term 0), -u (term 1)
        for (int c = 0; c < 3; ++c) {
            if (e_masked(c, i, j, k)) continue;
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
        for (int b = 0; b < 3; ++b)
            for (int s = 0; s < 2; ++s) {
                int w[3] = {i, j, k};
                w[b] -= s;
                U[b][s] = (double)(S * edge_at(d, eb[b], w[0], w[1], w[2]));
                Y[b][s] = (double)fwd_curl(d, b, w, fsr);
            }
        double G[3][3], A[3][3];
        for (int a = 0; a < 3; ++a) {
            G[a][a] = 0.5 * (U[a][0] * Y[a][0] + U[a][1] * Y[a][1]);
            for (int b = a + 1; b < 3; ++b) {
                const double g = 0.125 * ((U[a][0] + U[a][1]) * (Y[b][0] + Y[b][1]) +
                                          (U[b][0] + U[b][1]) * (Y[a][0] + Y[a][1]));
                G[a][b] = G[b][a] = g;
            }
            for (int b = 0; b < 3; ++b) A[a][b] = (double)tinv_at(d, tcomp(a, b), i, j, k);
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
void launch_tens_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, hipStream_t s) {
    const DomDev<T>* dp = (const DomDev<T>*)doms + dom;
    const dim3 grid((n[0] + kTx - 1) / kTx, (n[1] + kTy - 1) / kTy, std::min(n[2], kMaxGridZ));
    hipLaunchKernelGGL(k_tadj_ht<T>, grid, dim3(256), 0, s, dp, rs, ws);
    hipLaunchKernelGGL(k_tadj_e<T>, grid, dim3(256), 0, s, dp, rs, ws, fsr);
}

template void launch_tens_adj<float>(const void*, int, const int*, int, int, int, hipStream_t);
template void launch_tens_adj<double>(const void*, int, const int*, int, int, int, hipStream_t);

}  // namespace fdtd
