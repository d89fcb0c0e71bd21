// fdtd_kernels.hip -- HIP kernels of libfdtd for gfx950 (MI355X).
//
// The Yee step is memory bound (~1 flop per byte against a machine balance of
// ~20), so there is no matrix-core work here: kernels are organised around
// coalesced x-fastest rows, z-marching columns that keep the previous plane in
// registers, XCD-aware block placement and ping-ponged state.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
    int dom, i, j, k0, k1;
    bool ok;
};

// 256 threads = 64 (x) x 4 (y) columns; each marches a z chunk of length kz.
template <typename T>
__device__ __forceinline__ Col column(const DomDev<T>* doms, const int* bs, int ndom, int kz, const DomDev<T>*& dp) {
    Col c;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    c.dom = find_domain(bs, ndom, b);
    dp = doms + c.dom;
    const DomDev<T>& d = *dp;
    int lb = b - bs[c.dom];
    int nbx = (d.n[0] + 63) >> 6, nby = (d.n[1] + 3) >> 2;
    int bx = lb % nbx;
    int r = lb / nbx;
    int by = r % nby, bz = r / nby;
    c.i = bx * 64 + (threadIdx.x & 63);
    c.j = by * 4 + (threadIdx.x >> 6);
    c.k0 = bz * kz;
    c.k1 = min(c.k0 + kz, d.n[2]);
    c.ok = c.i < d.n[0] && c.j < d.n[1];
    return c;
}

// ============================================================ forward, split
template <typename T>
__global__ void __launch_bounds__(256) k_fwd_e(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                               int ndom, int kz, int p, int t) {
    const DomDev<T>* dp;
    Col c = column(doms, bs, ndom, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j;
    const T* Hx = d.H[p][0];
    const T* Hy = d.H[p][1];
    const T* Hz = d.H[p][2];
    T hxm = 0, hym = 0;   // Hx, Hy one plane below
    if (c.k0 > 0) {
        long long f = fidx(d, i, j, c.k0 - 1);
        hxm = Hx[f];
        hym = Hy[f];
    }
    for (int k = c.k0; k < c.k1; ++k) {
        long long f = fidx(d, i, j, k);
        T hx = Hx[f], hy = Hy[f], hz = Hz[f];
        T hy_xm = i > 0 ? Hy[f - 1] : T(0), hz_xm = i > 0 ? Hz[f - 1] : T(0);
        T hx_ym = j > 0 ? Hx[f - d.pitch] : T(0), hz_ym = j > 0 ? Hz[f - d.pitch] : T(0);
        // Ex: d-_y Hz - d-_z Hy ; Ey: d-_z Hx - d-_x Hz ; Ez: d-_x Hy - d-_y Hx
        T ex = e_update<T, true>(d, 0, i, j, k, f, hz, hz_ym, hy, hym, p, t);
        T ey = e_update<T, true>(d, 1, i, j, k, f, hx, hxm, hz, hz_xm, p, t);
        T ez = e_update<T, true>(d, 2, i, j, k, f, hy, hy_xm, hx, hx_ym, p, t);
        d.E[1 - p][0][f] = ex;
        d.E[1 - p][1][f] = ey;
        d.E[1 - p][2][f] = ez;
        hxm = hx;
        hym = hy;
    }
}

// reads E^{n+1} from set 1-p (written by k_fwd_e), H^{n+1/2} from set p
template <typename T>
__global__ void __launch_bounds__(256) k_fwd_h(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                               int ndom, int kz, int p) {
    const DomDev<T>* dp;
    Col c = column(doms, bs, ndom, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j, nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const T* Ex = d.E[1 - p][0];
    const T* Ey = d.E[1 - p][1];
    const T* Ez = d.E[1 - p][2];
    long long f0 = fidx(d, i, j, c.k0);
    T ex = Ex[f0], ey = Ey[f0], ez = Ez[f0];
    for (int k = c.k0; k < c.k1; ++k) {
        long long f = fidx(d, i, j, k);
        T ex1 = 0, ey1 = 0, ez1 = 0;
        if (k + 1 < nz) {
            ex1 = Ex[f + d.plane];
            ey1 = Ey[f + d.plane];
            ez1 = Ez[f + d.plane];
        }
        T ey_xp = i + 1 < nx ? Ey[f + 1] : T(0), ez_xp = i + 1 < nx ? Ez[f + 1] : T(0);
        T ex_yp = j + 1 < ny ? Ex[f + d.pitch] : T(0), ez_yp = j + 1 < ny ? Ez[f + d.pitch] : T(0);
        // Hx: d+_y Ez - d+_z Ey ; Hy: d+_z Ex - d+_x Ez ; Hz: d+_x Ey - d+_y Ex
        d.H[1 - p][0][f] = h_update(d, 0, i, j, k, f, ez_yp, ez, ey1, ey, p);
        d.H[1 - p][1][f] = h_update(d, 1, i, j, k, f, ex1, ex, ez_xp, ez, p);
        d.H[1 - p][2][f] = h_update(d, 2, i, j, k, f, ey_xp, ey, ex_yp, ex, p);
        ex = ex1;
        ey = ey1;
        ez = ez1;
    }
}

// ============================================================ adjoint, split
// H transpose: Et = Ebar + (d+)^T of the H-update terms, from Hbar (set p).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_ht(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                                int ndom, int kz, int p) {
    const DomDev<T>* dp;
    Col c = column(doms, bs, ndom, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    if (!d.grad) return;
    const int i = c.i, j = c.j;
    const T* Hx = d.Ha[p][0];
    const T* Hy = d.Ha[p][1];
    const T* Hz = d.Ha[p][2];
    T hxm = 0, hym = 0;
    if (c.k0 > 0) {
        long long f = fidx(d, i, j, c.k0 - 1);
        hxm = Hx[f];
        hym = Hy[f];
    }
    for (int k = c.k0; k < c.k1; ++k) {
        long long f = fidx(d, i, j, k);
        T hx = Hx[f], hy = Hy[f], hz = Hz[f];
        T hy_xm = i > 0 ? Hy[f - 1] : T(0), hz_xm = i > 0 ? Hz[f - 1] : T(0);
        T hx_ym = j > 0 ? Hx[f - d.pitch] : T(0), hz_ym = j > 0 ? Hz[f - d.pitch] : T(0);
        // Ebar_e: term 1 H_{e+1} along e+2 (+), term 2 H_{e+2} along e+1 (-)
        // Ex: Hy along z, Hz along y ; Ey: Hz along x, Hx along z ; Ez: Hx along y, Hy along x
        d.Et[0][f] = ht_update(d, 0, i, j, k, f, hy, hym, hz, hz_ym, p);
        d.Et[1][f] = ht_update(d, 1, i, j, k, f, hz, hz_xm, hx, hxm, p);
        d.Et[2][f] = ht_update(d, 2, i, j, k, f, hx, hx_ym, hy, hy_xm, p);
        hxm = hx;
        hym = hy;
    }
}

// Owner work at E node (i,j,k): E-update transposes of the three components,
// new cotangents of E^n and the memories, gradient from the forward state
// u^n (set fp), and the six raw-difference cotangents of the curl terms.
template <typename T>
struct Dbar6 {
    T x0, x1, y0, y1, z0, z1;   // component (x,y,z) term (0: along c+1, +; 1: along c+2, -)
};

template <typename T>
__device__ __forceinline__ Dbar6<T> et_owner(const DomDev<T>& d, int i, int j, int k, int p, int fp, bool in_g,
                                             double* gsum, double gc[3]) {
    long long f = fidx(d, i, j, k);
    Dbar6<T> o;
    T* dd[3][2] = {{&o.x0, &o.x1}, {&o.y0, &o.y1}, {&o.z0, &o.z1}};
    T H[3], Hm[3][3];   // forward H at the node and one step back along x, y, z
    if (in_g) {
        for (int q = 0; q < 3; ++q) H[q] = d.H[fp][q][f];
        for (int q = 0; q < 3; ++q) {
            Hm[0][q] = i > 0 ? d.H[fp][q][f - 1] : T(0);
            Hm[1][q] = j > 0 ? d.H[fp][q][f - d.pitch] : T(0);
            Hm[2][q] = k > 0 ? d.H[fp][q][f - d.plane] : T(0);
        }
    }
    for (int cc = 0; cc < 3; ++cc) {
        T et = d.Et[cc][f];
        AdjE<T> r = et_node<T, true>(d, cc, i, j, k, f, et, p);
        d.Ea[1 - p][cc][f] = r.en;
        const int a0 = (cc + 1) % 3, a1 = (cc + 2) % 3;
        if (e_masked(cc, i, j, k)) {
            *dd[cc][0] = T(0);
            *dd[cc][1] = T(0);
            continue;
        }
        *dd[cc][0] = et_dbar<T, true>(d, a0, 0, T(1), i, j, k, r.epre, r.coef, p);
        *dd[cc][1] = et_dbar<T, true>(d, a1, 1, T(-1), i, j, k, r.epre, r.coef, p);
        if (in_g) {
            const int h0 = (cc + 2) % 3, h1 = (cc + 1) % 3;
            T curl = curl_minus_ro(d, cc, i, j, k, H[h0], Hm[a0][h0], H[h1], Hm[a1][h1], fp);
            T einv = epsinv_at(d, cc, i, j, k);
            double g;
            if (in_lor(d, i, j, k)) {
                long long q = lidx(d, i, j, k);
                T e = d.E[fp][cc][f];
                T eold = d.lor[fp][0][cc][q], w = d.lor[fp][1][cc][q], wold = d.lor[fp][2][cc][q];
                T einf = T(1) / einv;
                T invden = T(1) / (einf + T(0.25) * d.lg);
                T num = fma(einf, e, T(0.25) * d.lg * eold);
                num = fma(d.S, curl, num);
                num -= T(0.5) * fma(T(1) + d.lal, w, d.lxi * wold);
                T epre_f = num * invden;
                g = (double)r.epre * (double)((e - epre_f) * invden);
            } else {
                g = -(double)r.epre * (double)(d.S * einv * einv * curl);
            }
            gc[cc] = g;
            *gsum += g;
        }
    }
    return o;
}

template <typename T>
__device__ __forceinline__ bool in_gbox(const DomDev<T>& d, int i, int j, int k) {
    return i >= d.glo[0] && i < d.ghi[0] && j >= d.glo[1] && j < d.ghi[1] && k >= d.glo[2] && k < d.ghi[2];
}

template <typename T>
__device__ __forceinline__ void grad_store(const DomDev<T>& d, int i, int j, int k, double gsum, const double gc[3]) {
    long long q = ((long long)(k - d.glo[2]) * (d.ghi[1] - d.glo[1]) + (j - d.glo[1])) * (d.ghi[0] - d.glo[0]) +
                  (i - d.glo[0]);
    if (d.eps_diag) {
        d.gacc[0][q] += gc[0];
        d.gacc[1][q] += gc[1];
        d.gacc[2][q] += gc[2];
    } else {
        d.gacc[0][q] += gsum;
    }
}

// Raw-difference cotangent of one curl term at a neighbouring E node, read only.
template <typename T>
__device__ __forceinline__ T et_dbar_at(const DomDev<T>& d, int cc, int term, int i, int j, int k, int p) {
    if (e_masked(cc, i, j, k)) return T(0);
    long long f = fidx(d, i, j, k);
    AdjE<T> r = et_node<T, false>(d, cc, i, j, k, f, d.Et[cc][f], p);
    int a = term == 0 ? (cc + 1) % 3 : (cc + 2) % 3;
    return et_dbar<T, false>(d, a, term, term == 0 ? T(1) : T(-1), i, j, k, r.epre, r.coef, p);
}

// E transpose: Hbar += (d-)^T of the E-update terms; owner updates at E nodes.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_et(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                                int ndom, int kz, int p, int fp) {
    const DomDev<T>* dp;
    Col c = column(doms, bs, ndom, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    if (!d.grad) return;
    const int i = c.i, j = c.j, nx = d.n[0], ny = d.n[1], nz = d.n[2];
    double gsum = 0, gc[3] = {0, 0, 0};
    bool ing = in_gbox(d, i, j, c.k0);
    Dbar6<T> cur = et_owner(d, i, j, c.k0, p, fp, ing, &gsum, gc);
    if (ing) grad_store(d, i, j, c.k0, gsum, gc);
    for (int k = c.k0; k < c.k1; ++k) {
        long long f = fidx(d, i, j, k);
        // z-terms one plane up: Ey term 0 (along z), Ex term 1 (along z)
        Dbar6<T> nxt{};
        T up_y0 = 0, up_x1 = 0;
        if (k + 1 < c.k1) {
            gsum = 0;
            gc[0] = gc[1] = gc[2] = 0;
            ing = in_gbox(d, i, j, k + 1);
            nxt = et_owner(d, i, j, k + 1, p, fp, ing, &gsum, gc);
            if (ing) grad_store(d, i, j, k + 1, gsum, gc);
            up_y0 = nxt.y0;
            up_x1 = nxt.x1;
        } else if (k + 1 < nz) {
            up_y0 = et_dbar_at(d, 1, 0, i, j, k + 1, p);
            up_x1 = et_dbar_at(d, 0, 1, i, j, k + 1, p);
        }
        // x neighbour: Ez term 0 and Ey term 1 (along x); y neighbour: Ez term 1, Ex term 0 (along y)
        T xp_z0 = 0, xp_y1 = 0, yp_z1 = 0, yp_x0 = 0;
        if (i + 1 < nx) {
            xp_z0 = et_dbar_at(d, 2, 0, i + 1, j, k, p);
            xp_y1 = et_dbar_at(d, 1, 1, i + 1, j, k, p);
        }
        if (j + 1 < ny) {
            yp_z1 = et_dbar_at(d, 2, 1, i, j + 1, k, p);
            yp_x0 = et_dbar_at(d, 0, 0, i, j + 1, k, p);
        }
        T hbx = d.Ha[p][0][f], hby = d.Ha[p][1][f], hbz = d.Ha[p][2][f];
        // memory cotangents of the H update at this node (input Hbar)
        hT_dbar<T, true>(d, 1, 0, T(1), i, j, k, hbx, p);   // Hx term 0 along y
        hT_dbar<T, true>(d, 2, 1, T(-1), i, j, k, hbx, p);  // Hx term 1 along z
        hT_dbar<T, true>(d, 2, 0, T(1), i, j, k, hby, p);   // Hy term 0 along z
        hT_dbar<T, true>(d, 0, 1, T(-1), i, j, k, hby, p);  // Hy term 1 along x
        hT_dbar<T, true>(d, 0, 0, T(1), i, j, k, hbz, p);   // Hz term 0 along x
        hT_dbar<T, true>(d, 1, 1, T(-1), i, j, k, hbz, p);  // Hz term 1 along y
        hbx += (cur.y0 - up_y0) + (cur.z1 - yp_z1);
        hby += (cur.z0 - xp_z0) + (cur.x1 - up_x1);
        hbz += (cur.x0 - yp_x0) + (cur.y1 - xp_y1);
        d.Ha[1 - p][0][f] = hbx;
        d.Ha[1 - p][1][f] = hby;
        d.Ha[1 - p][2][f] = hbz;
        cur = nxt;
    }
}

// ============================================================ monitors
// Sample one plane monitor into slot `slot` of its ring buffer
// [block][ncomp][npts] (E at time n, H at n + 1/2; flux H averaged over
// planes k and k-1).
template <typename T>
__global__ void k_sample(const DomDev<T>* __restrict__ doms, MonDev m, int p, int slot) {
    const DomDev<T>& d = doms[m.dom];
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int ni = m.i1 - m.i0, npts = ni * (m.j1 - m.j0);
    if (q >= npts) return;
    int i = m.i0 + q % ni, j = m.j0 + q / ni, k = m.k;
    long long f = fidx(d, i, j, k);
    T* buf = (T*)m.samples + (long long)slot * m.ncomp * npts;
    if (m.kind == 1) {
        T hxm = k > 0 ? d.H[p][0][f - d.plane] : T(0);
        T hym = k > 0 ? d.H[p][1][f - d.plane] : T(0);
        buf[q] = d.E[p][0][f];
        buf[npts + q] = d.E[p][1][f];
        buf[2 * npts + q] = T(0.5) * (d.H[p][0][f] + hxm);
        buf[3 * npts + q] = T(0.5) * (d.H[p][1][f] + hym);
    } else {
        buf[q] = m.comp < 3 ? d.E[p][m.comp][f] : d.H[p][m.comp - 3][f];
    }
}

// Accumulate `count` buffered samples taken at steps n0 .. n0+count-1 into the
// FP64 spectra acc[f][comp][pt] += x * exp(-i w t), t = n (E) or n + 1/2 (H).
// grid.y = frequency; the block's twiddles sit in LDS.
template <typename T>
__global__ void k_dft(MonDev m, int n0, int count) {
    __shared__ double tw[2][2][kMaxDftBlock];   // [E|H][cos|sin][sample]
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
        double re = 0, im = 0;
        for (int s = 0; s < count; ++s) {
            double x = (double)buf[((long long)s * m.ncomp + cq) * npts + q];
            re = fma(x, tw[ish][0][s], re);
            im = fma(-x, tw[ish][1][s], im);
        }
        double* a = m.acc + (((long long)f * m.ncomp + cq) * npts + q) * 2;
        a[0] += re;
        a[1] += im;
    }
}

template <typename T>
__global__ void k_probe(const DomDev<T>* __restrict__ doms, MonDev m, int p, int n) {
    const DomDev<T>& d = doms[m.dom];
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long f = fidx(d, m.pi, m.pj, m.k);
        m.trace[n] = (double)(m.comp < 3 ? d.E[p][m.comp][f] : d.H[p][m.comp - 3][f]);
    }
}

// Seeds dJ/du^n of one plane monitor into the cotangent state (set p):
// Re sum_f G_f exp(+i w t), t = n (E) or n + 1/2 (H).
template <typename T>
__global__ void k_seed(const DomDev<T>* __restrict__ doms, MonDev m, int p, int n) {
    const DomDev<T>& d = doms[m.dom];
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    int ni = m.i1 - m.i0;
    int i = m.i0 + q % ni, j = m.j0 + q / ni, k = m.k;
    long long f = fidx(d, i, j, k);
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
            T* H = d.Ha[p][comp - 3];
            H[f] += (T)(0.5 * s);
            if (k > 0) H[f - d.plane] += (T)(0.5 * s);
        } else if (ish) {
            d.Ha[p][comp - 3][f] += (T)s;
        } else {
            d.Ea[p][comp][f] += (T)s;
        }
    }
}

template <typename T>
__global__ void k_probe_seed(const DomDev<T>* __restrict__ doms, MonDev m, int p, int n) {
    const DomDev<T>& d = doms[m.dom];
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long f = fidx(d, m.pi, m.pj, m.k);
        double g = m.cot[n - 1];
        if (m.comp < 3) d.Ea[p][m.comp][f] += (T)g;
        else d.Ha[p][m.comp - 3][f] += (T)g;
    }
}

// ============================================================ utilities
__global__ void k_fill_zero(uint32_t* __restrict__ p, long long n_words) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; q < n_words; q += stride) p[q] = 0u;
}

// max |x| of an FP32 array into *out (as ordered bits; out pre-zeroed)
__global__ void k_maxabs_f32(const float* __restrict__ x, long long n, unsigned int* out) {
    float m = 0.f;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[q]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// x / scale rounded to bfloat16 (round to nearest even)
__global__ void k_pack_bf16(const float* __restrict__ x, long long n, const unsigned int* scale_bits,
                            uint16_t* __restrict__ y) {
    float s = __uint_as_float(*scale_bits);
    float inv = s > 0.f ? 1.f / s : 0.f;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        uint32_t u = __float_as_uint(x[q] * inv);
        uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
        y[q] = (uint16_t)(r >> 16);
    }
}

__global__ void k_unpack_bf16(const uint16_t* __restrict__ y, long long n, const unsigned int* scale_bits,
                              float* __restrict__ x) {
    float s = __uint_as_float(*scale_bits);
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        x[q] = __uint_as_float(((uint32_t)y[q]) << 16) * s;
}

// 64-bit wrap-around sum of 32-bit words (slot checksum)
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

template <typename T>
void launch_fwd_split(const void* doms, const int* bs, int ndom, int nblocks, int kz, int p, int t, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd_e<T>, dim3(nblocks), dim3(256), 0, s, (const DomDev<T>*)doms, bs, ndom, kz, p, t);
    hipLaunchKernelGGL(k_fwd_h<T>, dim3(nblocks), dim3(256), 0, s, (const DomDev<T>*)doms, bs, ndom, kz, p);
}

template <typename T>
void launch_adj_split(const void* doms, const int* bs, int ndom, int nblocks, int kz, int p, int fp, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_ht<T>, dim3(nblocks), dim3(256), 0, s, (const DomDev<T>*)doms, bs, ndom, kz, p);
    hipLaunchKernelGGL(k_adj_et<T>, dim3(nblocks), dim3(256), 0, s, (const DomDev<T>*)doms, bs, ndom, kz, p, fp);
}

template <typename T>
void launch_sample(const void* doms, const MonDev& m, int p, int slot, hipStream_t s) {
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_sample<T>, dim3((npts + 255) / 256), dim3(256), 0, s, (const DomDev<T>*)doms, m, p, slot);
}

template <typename T>
void launch_dft(const MonDev& m, int n0, int count, hipStream_t s) {
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_dft<T>, dim3((npts + 255) / 256, m.nf), dim3(256), 0, s, m, n0, count);
}

template <typename T>
void launch_probe(const void* doms, const MonDev& m, int p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_probe<T>, dim3(1), dim3(64), 0, s, (const DomDev<T>*)doms, m, p, n);
}

template <typename T>
void launch_seed(const void* doms, const MonDev& m, int p, int n, hipStream_t s) {
    if (m.kind == 0) {
        hipLaunchKernelGGL(k_probe_seed<T>, dim3(1), dim3(64), 0, s, (const DomDev<T>*)doms, m, p, n);
        return;
    }
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_seed<T>, dim3((npts + 255) / 256), dim3(256), 0, s, (const DomDev<T>*)doms, m, p, n);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    long long nw = (long long)(bytes / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_1d(nw, 256, 8192)), dim3(256), 0, s, (uint32_t*)p, nw);
}

void launch_maxabs_f32(const float* x, long long n, unsigned int* out, hipStream_t s) {
    hipLaunchKernelGGL(k_maxabs_f32, dim3(blocks_1d(n, 256, 4096)), dim3(256), 0, s, x, n, out);
}

void launch_pack_bf16(const float* x, long long n, const unsigned int* scale, uint16_t* y, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_bf16, dim3(blocks_1d(n, 256, 8192)), dim3(256), 0, s, x, n, scale, y);
}

void launch_unpack_bf16(const uint16_t* y, long long n, const unsigned int* scale, float* x, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack_bf16, dim3(blocks_1d(n, 256, 8192)), dim3(256), 0, s, y, n, scale, x);
}

void launch_checksum(const void* p, size_t bytes, unsigned long long* out, hipStream_t s) {
    long long nw = (long long)(bytes / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_checksum, dim3(blocks_1d(nw, 256, 4096)), dim3(256), 0, s, (const uint32_t*)p, nw, out);
}

#define FDTD_INSTANTIATE(T)                                                                                      \
    template void launch_fwd_split<T>(const void*, const int*, int, int, int, int, int, hipStream_t);            \
    template void launch_adj_split<T>(const void*, const int*, int, int, int, int, int, hipStream_t);            \
    template void launch_sample<T>(const void*, const MonDev&, int, int, hipStream_t);                           \
    template void launch_dft<T>(const MonDev&, int, int, hipStream_t);                                           \
    template void launch_probe<T>(const void*, const MonDev&, int, int, hipStream_t);                            \
    template void launch_seed<T>(const void*, const MonDev&, int, int, hipStream_t);
FDTD_INSTANTIATE(float)
FDTD_INSTANTIATE(double)

}  // namespace fdtd
