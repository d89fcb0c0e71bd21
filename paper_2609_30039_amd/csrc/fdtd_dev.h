// fdtd_dev.h -- device-side data layout and per-node arithmetic of libfdtd.
//
// Layout (per domain):
//   fields         E[set][c], H[set][c]: [nz][ny][pitch], x fastest, pitch a
//                  multiple of 128 B so every row starts on a cache line;
//   absorbers      psi slabs per face (axis a, side s) for the two components
//                  that take a-derivatives; x faces [nz][ny][L], y faces
//                  [nz][L][nx], z faces [L][ny][nx];
//   material       eps^-1 over a box (one array for isotropic media, three for
//                  diagonal tensors), a scalar outside;
//   Lorentz        E^{n-1}, W^n, W^{n-1} per component over the Lorentz box.
// Every quantity that a neighbouring tile may read during a step is kept in
// two sets (ping-pong): a step reads set p and writes set 1-p, so tiles can
// recompute halos without ordering constraints between workgroups.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtd {

constexpr int kMaxSrc = 4;

template <typename T>
struct SrcDev {
    int kind, comp, i, j, k, nwave;
    const T* wave;
};

template <typename T>
struct DomDev {
    int n[3];                  // cells along x, y, z
    int pitch;                 // row pitch of field arrays
    long long plane;           // pitch * ny
    T S;
    // ---- forward state ----
    T* E[2][3];
    T* H[2][3];
    int L[3][2];               // absorbing depth per axis and side
    const T* tab[3];           // per axis 6 tables of n[a]: bE cE kiE bH cH kiH
    T* psiE[2][3][2][2];       // [set][axis][side][r], r = 0 -> component (a+2)%3, 1 -> (a+1)%3
    T* psiH[2][3][2][2];
    int eps_diag;
    int elo[3], ehi[3];
    T epsinv_bg;
    const T* epsinv[3];        // over the eps box; isotropic: the same array thrice
    int has_lor;
    int llo[3], lhi[3];
    T lal, lxi, lg;            // pole recursion constants
    T* lor[2][3][3];           // [set][0 Eold | 1 W | 2 Wold][component] over the Lorentz box
    int nsrc;
    SrcDev<T> src[kMaxSrc];
    // ---- adjoint state ----
    int grad;                  // domain takes part in the adjoint
    T* Ea[2][3];
    T* Ha[2][3];
    T* Et[3];                  // split transpose: cotangent of E^{n+1} after the H transpose
    T* psiEa[2][3][2][2];
    T* psiHa[2][3][2][2];
    T* lora[2][3][3];
    int glo[3], ghi[3];
    double* gacc[3];           // dJ/deps accumulators over the gradient box (isotropic: [0] only)
};

// ------------------------------------------------------------------ indexing
template <typename T>
__device__ __forceinline__ long long fidx(const DomDev<T>& d, int i, int j, int k) {
    return (long long)k * d.plane + (long long)j * d.pitch + i;
}

// side of the absorbing slab containing index x along axis a: 0 low, 1 high, -1 none
template <typename T>
__device__ __forceinline__ int slab_side(const DomDev<T>& d, int a, int x) {
    if (x < d.L[a][0]) return 0;
    if (x >= d.n[a] - d.L[a][1]) return 1;
    return -1;
}

template <typename T>
__device__ __forceinline__ long long pidx(const DomDev<T>& d, int a, int s, int i, int j, int k) {
    int L = d.L[a][s];
    if (a == 0) {
        int ii = s ? i - (d.n[0] - L) : i;
        return ((long long)k * d.n[1] + j) * L + ii;
    }
    if (a == 1) {
        int jj = s ? j - (d.n[1] - L) : j;
        return ((long long)k * L + jj) * d.n[0] + i;
    }
    int kk = s ? k - (d.n[2] - L) : k;
    return ((long long)kk * d.n[1] + j) * d.n[0] + i;
}

template <typename T>
__device__ __forceinline__ T epsinv_at(const DomDev<T>& d, int c, int i, int j, int k) {
    if (i >= d.elo[0] && i < d.ehi[0] && j >= d.elo[1] && j < d.ehi[1] && k >= d.elo[2] && k < d.ehi[2]) {
        long long q = ((long long)(k - d.elo[2]) * (d.ehi[1] - d.elo[1]) + (j - d.elo[1])) * (d.ehi[0] - d.elo[0]) +
                      (i - d.elo[0]);
        return d.epsinv[c][q];
    }
    return d.epsinv_bg;
}

template <typename T>
__device__ __forceinline__ bool in_lor(const DomDev<T>& d, int i, int j, int k) {
    return d.has_lor && i >= d.llo[0] && i < d.lhi[0] && j >= d.llo[1] && j < d.lhi[1] && k >= d.llo[2] &&
           k < d.lhi[2];
}

template <typename T>
__device__ __forceinline__ long long lidx(const DomDev<T>& d, int i, int j, int k) {
    return ((long long)(k - d.llo[2]) * (d.lhi[1] - d.llo[1]) + (j - d.llo[1])) * (d.lhi[0] - d.llo[0]) +
           (i - d.llo[0]);
}

__device__ __forceinline__ int coord(int a, int i, int j, int k) { return a == 0 ? i : (a == 1 ? j : k); }

// PEC: E_c is held at zero where the index along c+1 or c+2 is 0
__device__ __forceinline__ bool e_masked(int c, int i, int j, int k) {
    return coord((c + 1) % 3, i, j, k) == 0 || coord((c + 2) % 3, i, j, k) == 0;
}

// ---------------------------------------------------------- forward pieces
// Stretched difference for one curl term: D raw difference along axis a at
// node (i,j,k), r the slab component slot.  tab offset 0 (E side) or 3 (H side).
template <typename T, bool WRITE>
__device__ __forceinline__ T stretch(const DomDev<T>& d, T* const (&psi)[2][3][2][2], int p, int a, int r, int toff,
                                     int i, int j, int k, T D) {
    int x = coord(a, i, j, k);
    int s = slab_side(d, a, x);
    if (s < 0) return D;
    const T* tb = d.tab[a];
    int n = d.n[a];
    T b = tb[(toff + 0) * n + x], c = tb[(toff + 1) * n + x], ki = tb[(toff + 2) * n + x];
    long long q = pidx(d, a, s, i, j, k);
    T pn = fma(b, psi[p][a][s][r][q], c * D);
    if (WRITE) psi[1 - p][a][s][r][q] = pn;
    return fma(ki, D, pn);
}

// New E_c at node (i,j,k) from H^{n+1/2} (set p): h0 = H_{c+2} at the node and
// h0m one step back along a0 = c+1; h1 = H_{c+1} and h1m back along a1 = c+2.
// With WRITE the absorber memories and Lorentz history of set 1-p are
// written (the owning tile); without, the value is only recomputed (halo).
template <typename T, bool WRITE>
__device__ __forceinline__ T e_update(const DomDev<T>& d, int c, int i, int j, int k, long long f, T h0, T h0m,
                                      T h1, T h1m, int p, int t) {
    const bool lorc = in_lor(d, i, j, k);
    if (e_masked(c, i, j, k)) {
        if (WRITE && lorc) {
            long long q = lidx(d, i, j, k);
            d.lor[1 - p][0][c][q] = T(0);
            d.lor[1 - p][1][c][q] = T(0);
            d.lor[1 - p][2][c][q] = T(0);
        }
        return T(0);
    }
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch<T, WRITE>(d, d.psiE, p, a0, 0, 0, i, j, k, h0 - h0m);
    T D1 = stretch<T, WRITE>(d, d.psiE, p, a1, 1, 0, i, j, k, h1 - h1m);
    T curl = D0 - D1;
    T einv = epsinv_at(d, c, i, j, k);
    T e = d.E[p][c][f];
    T en;
    long long q = 0;
    T eold = 0, w = 0, wold = 0;
    if (lorc) {
        q = lidx(d, i, j, k);
        eold = d.lor[p][0][c][q];
        w = d.lor[p][1][c][q];
        wold = d.lor[p][2][c][q];
        T einf = T(1) / einv;
        T invden = T(1) / (einf + T(0.25) * d.lg);
        T num = fma(einf, e, T(0.25) * d.lg * eold);
        num = fma(d.S, curl, num);
        num -= T(0.5) * fma(T(1) + d.lal, w, d.lxi * wold);
        en = num * invden;
    } else {
        en = fma(d.S * einv, curl, e);
    }
    for (int s = 0; s < d.nsrc; ++s) {
        const SrcDev<T>& sr = d.src[s];
        if (sr.comp == c && t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j))) en += sr.wave[t];
    }
    if (WRITE && lorc) {
        T wn = fma(d.lal, w, d.lxi * wold);
        wn = fma(T(0.5) * d.lg, en - eold, wn);
        d.lor[1 - p][0][c][q] = e;
        d.lor[1 - p][1][c][q] = wn;
        d.lor[1 - p][2][c][q] = w;
    }
    return en;
}

// New H_c at node (i,j,k) from E^{n+1}: e0p/e0 = E_{c+2} one step forward along
// a0 = c+1 and at the node; e1p/e1 = E_{c+1} forward along a1 = c+2.
template <typename T>
__device__ __forceinline__ T h_update(const DomDev<T>& d, int c, int i, int j, int k, long long f, T e0p, T e0,
                                      T e1p, T e1, int p) {
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch<T, true>(d, d.psiH, p, a0, 0, 3, i, j, k, e0p - e0);
    T D1 = stretch<T, true>(d, d.psiH, p, a1, 1, 3, i, j, k, e1p - e1);
    return fma(-d.S, D0 - D1, d.H[p][c][f]);
}

// Stretched backward-difference curl of the forward H (set p) at E node,
// read-only (the gradient needs it from u^n without touching the state).
template <typename T>
__device__ __forceinline__ T curl_minus_ro(const DomDev<T>& d, int c, int i, int j, int k, T h0, T h0m, T h1, T h1m,
                                           int p) {
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch<T, false>(d, d.psiE, p, a0, 0, 0, i, j, k, h0 - h0m);
    T D1 = stretch<T, false>(d, d.psiE, p, a1, 1, 0, i, j, k, h1 - h1m);
    return D0 - D1;
}

// ---------------------------------------------------------- adjoint pieces
// Transposed absorber recursion (Section 3.1): from the cotangent ybar of the
// stretched derivative and the memory cotangent psibar, the cotangent of the
// raw difference is ki*ybar + c*(psibar + ybar) and the memory cotangent
// becomes b*(psibar + ybar).
template <typename T, bool WRITE>
__device__ __forceinline__ T stretch_T(const DomDev<T>& d, T* const (&psi)[2][3][2][2], int p, int a, int r,
                                       int toff, int i, int j, int k, T ybar) {
    int x = coord(a, i, j, k);
    int s = slab_side(d, a, x);
    if (s < 0) return ybar;
    const T* tb = d.tab[a];
    int n = d.n[a];
    T b = tb[(toff + 0) * n + x], c = tb[(toff + 1) * n + x], ki = tb[(toff + 2) * n + x];
    long long q = pidx(d, a, s, i, j, k);
    T mem = psi[p][a][s][r][q] + ybar;
    if (WRITE) psi[1 - p][a][s][r][q] = b * mem;
    return fma(ki, ybar, c * mem);
}

// Cotangent of the raw forward difference d+_a E of the H_h update term
// (a, sign, r) at H node (i,j,k): ybar = -S sign Hbar_h.
template <typename T, bool WRITE>
__device__ __forceinline__ T hT_dbar(const DomDev<T>& d, int a, int r, T sgn, int i, int j, int k, T hbar, int p) {
    return stretch_T<T, WRITE>(d, d.psiHa, p, a, r, 3, i, j, k, -d.S * sgn * hbar);
}

// H transpose at E node: Ebar_e after adding (d+)^T of the two H terms that
// differentiate E_e.  Term 1: H_{e+1} along e+2, sign +, slot r=0;
// term 2: H_{e+2} along e+1, sign -, slot r=1.  hb1/hb1m: H_{e+1} cotangent at
// the node and one step back along e+2; hb2/hb2m likewise along e+1.
template <typename T>
__device__ __forceinline__ T ht_update(const DomDev<T>& d, int e, int i, int j, int k, long long f, T hb1, T hb1m,
                                       T hb2, T hb2m, int p) {
    if (e_masked(e, i, j, k)) return T(0);
    const int a1 = (e + 2) % 3, a2 = (e + 1) % 3;
    T acc = d.Ea[p][e][f];
    T t1 = hT_dbar<T, false>(d, a1, 0, T(1), i, j, k, hb1, p);
    T t1m = coord(a1, i, j, k) > 0
                ? hT_dbar<T, false>(d, a1, 0, T(1), i - (a1 == 0), j - (a1 == 1), k - (a1 == 2), hb1m, p)
                : T(0);
    T t2 = hT_dbar<T, false>(d, a2, 1, T(-1), i, j, k, hb2, p);
    T t2m = coord(a2, i, j, k) > 0
                ? hT_dbar<T, false>(d, a2, 1, T(-1), i - (a2 == 0), j - (a2 == 1), k - (a2 == 2), hb2m, p)
                : T(0);
    acc += t1m - t1;
    acc += t2m - t2;
    return acc;
}

// E-update transpose at E node c.  From etot (cotangent of E^{n+1} after the
// H transpose) returns the cotangent of E^{n+1} before the source, epre, and
// the coefficient that multiplies the curl (eps^-1 or 1/den).  With OWNER the
// Lorentz history transpose is applied to set 1-p, the new cotangent of E^n
// is returned in en, and the gradient contribution in dg (needs the forward
// state: curl of H^{n+1/2} and, for Lorentz nodes, E^n, E^{n-1}, W^n, W^{n-1}
// of set fp).
template <typename T>
struct AdjE {
    T epre, coef, en;
};

template <typename T, bool OWNER>
__device__ __forceinline__ AdjE<T> et_node(const DomDev<T>& d, int c, int i, int j, int k, long long f, T etot,
                                           int p) {
    AdjE<T> r;
    r.epre = T(0);
    r.coef = T(0);
    r.en = T(0);
    if (e_masked(c, i, j, k)) {
        if (OWNER && in_lor(d, i, j, k)) {
            long long q = lidx(d, i, j, k);
            d.lora[1 - p][0][c][q] = T(0);
            d.lora[1 - p][1][c][q] = T(0);
            d.lora[1 - p][2][c][q] = T(0);
        }
        return r;
    }
    T einv = epsinv_at(d, c, i, j, k);
    if (in_lor(d, i, j, k)) {
        long long q = lidx(d, i, j, k);
        T wb = d.lora[p][1][c][q];
        T einf = T(1) / einv;
        T invden = T(1) / (einf + T(0.25) * d.lg);
        T ep = fma(T(0.5) * d.lg, wb, etot);      // W^{n+1} roll feeds E^{n+1}
        r.epre = ep;
        r.coef = invden;
        if (OWNER) {
            T wob = d.lora[p][2][c][q], eob = d.lora[p][0][c][q];
            T wn = fma(d.lal, wb, wob);
            T wnm1 = d.lxi * wb;
            T enm1 = -T(0.5) * d.lg * wb;
            T s = ep * invden;
            r.en = fma(einf, s, eob);
            enm1 = fma(T(0.25) * d.lg, s, enm1);
            wn = fma(-T(0.5) * (T(1) + d.lal), s, wn);
            wnm1 = fma(-T(0.5) * d.lxi, s, wnm1);
            d.lora[1 - p][0][c][q] = enm1;
            d.lora[1 - p][1][c][q] = wn;
            d.lora[1 - p][2][c][q] = wnm1;
        }
    } else {
        r.epre = etot;
        r.coef = einv;
        r.en = etot;
    }
    return r;
}

// Cotangent of the raw backward difference d-_a H of the E_c update term
// (a, sign, r) at E node: ybar = S coef sign Ebar_pre.
template <typename T, bool WRITE>
__device__ __forceinline__ T et_dbar(const DomDev<T>& d, int a, int r, T sgn, int i, int j, int k, T epre, T coef,
                                     int p) {
    return stretch_T<T, WRITE>(d, d.psiEa, p, a, r, 0, i, j, k, d.S * coef * sgn * epre);
}

}  // namespace fdtd
