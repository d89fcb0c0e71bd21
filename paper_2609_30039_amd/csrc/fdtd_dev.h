// fdtd_dev.h -- device-side data layout and per-node arithmetic of libfdtd.
//
// Layout (per domain):
//   fields         E[c], H[c]: [nz][ny][pitch], x fastest, pitch a multiple of
//                  128 B so every row starts on a cache line;
//   absorbers      psi slabs per face (axis a, side s) for the two components
//                  that take a-derivatives; x faces [nz][ny][L], y faces
//                  [nz][L][nx], z faces [L][ny][nx];
//   material       eps^-1 over a box (one array for isotropic media, three for
//                  diagonal tensors), a scalar outside;
//   Lorentz        E^{n-1}, W^n, W^{n-1} per component over the Lorentz box.
// The forward state of all domains forms one "state set"; state sets are
// laid out at a fixed stride fs (elements), so the pointers stored here are
// those of set 0 and set q lives at +q*fs.  Sets 0 and 1 are working sets; a
// step reads one set and writes another, so tiles can recompute halos without
// ordering between workgroups, and checkpoint slots are further sets that a
// step can read directly.  The adjoint state has its own two sets (stride as).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtd {

constexpr int kMaxSrc = 4;
constexpr int kMaxPole = 16;
constexpr int kMaxSmp = 8;   // plane monitors per domain (the descriptor limit)

// A plane monitor as the split H kernel samples it: the threads whose column
// lies in the rectangle write their node's values into slot `slot` of the ring
// [block][rcomp][npts].  Flux rings hold Ex, Ey (plane k), Hx at k and k-1, Hy
// at k and k-1; the spectrum update averages the two H planes.
struct SmpDev {
    int kind;                  // 1 flux, 2 patch
    int comp;                  // patch component 0..5
    int i0, i1, j0, j1, k;
    int npts, rcomp;
    void* ring;
};

// Global-address-space views of device pointers.  Pointers read out of a
// descriptor are generic to the compiler, which would emit flat memory
// instructions; flat loads also count against the LDS wait counter, so a
// barrier's LDS wait would drain every prefetched global load.
#define FDTD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ FDTD_GLOBAL T* gp(T* p) {
    return (FDTD_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const FDTD_GLOBAL T* gp(const T* p) {
    return (const FDTD_GLOBAL T*)p;
}

// streaming store: the written field is not read again by this launch
template <typename T>
__device__ __forceinline__ void st_nt(FDTD_GLOBAL T* p, int off, T v) {
    __builtin_nontemporal_store(v, p + off);
}

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
    long long fs, as;          // forward / adjoint state-set strides (elements)
    // ---- forward state (set 0) ----
    T* E[3];
    T* H[3];
    int L[3][2];               // absorbing depth per axis and side
    const T* tab[3];           // per axis 6 tables of n[a]: bE cE kiE bH cH kiH
    T* psiE[3][2][2];          // [axis][side][r], r = 0 -> component (a+2)%3, 1 -> (a+1)%3
    T* psiH[3][2][2];
    int eps_diag;
    int elo[3], ehi[3];
    // rows of the stored eps box: x from exa (elo[0] rounded down to a 128-byte
    // boundary of the field rows) over exs elements (a multiple of 128 bytes), so
    // that a wave's eps^-1 loads touch the cache lines its field loads do
    int exa, exs;
    T epsinv_bg;
    const T* epsinv[3];        // over the eps box; isotropic: the same array thrice
    // symmetric tensor media (Section 2.3): eps^-1 at the grid nodes of the
    // eps box, six arrays xx yy zz xy xz yz over [elo, ehi) (the background
    // times the identity elsewhere); curl: the stretched curl of every E edge
    // of the current step, written by the first E pass, read by the assembly
    int tens;
    const T* tinv[6];
    T* curl[3];
    int onep;                  // the domain's interior blocks may take the single-pass kernel
    int has_lor;
    int llo[3], lhi[3];
    int npole;                 // poles of the dispersive box (1..kMaxPole)
    T lal[kMaxPole], lxi[kMaxPole], lg[kMaxPole];   // per-pole recursion constants
    T lgs;                     // sum of lg: the E^{n-1} weight, denominator eps + lgs/4
    long long lbox;            // cells of the box: pole p of W and Wold at + p * lbox
    T* lor[3][3];              // [0 Eold | 1 W | 2 Wold][component] over the Lorentz box
    // Bloch-periodic axes (Section 2.2; x and y only): no wall, and the
    // neighbour past the last node is the first one times bsign (+1 or -1)
    int per[3];
    T bsign[3];
    int nsrc;
    SrcDev<T> src[kMaxSrc];
    int nsmp;                  // plane monitors sampled inside the split H kernel
    SmpDev smp[kMaxSmp];
    // ---- adjoint state (set 0) ----
    int grad;                  // domain takes part in the adjoint
    T* Ea[3];
    T* Ha[3];
    T* Et[3];                  // split transpose: cotangent of E^{n+1} after the H transpose
    T* psiEa[3][2][2];
    T* psiHa[3][2][2];
    T* lora[3][3];
    int glo[3], ghi[3];
    double* gacc[6];           // dJ/deps accumulators over the gradient box: [0] isotropic, [0..2]
                               // diagonal, [0..5] the stored entries of a node tensor
    // ---- reversible mode: the lossless box R = [rlo, rhi) (the cells outside
    // every absorbing slab) is stepped backward; rec holds, per forward step
    // index, the fields just outside R that its backward steps need: H on the
    // three low faces (index rlo_a - 1) and E on the three high faces (rhi_a),
    // the two components tangential to the face, [face][comp][cells]
    int rev;
    int rlo[3], rhi[3];
    T* rec;
    long long rec_stride;      // elements per recorded step
    long long rface[6];        // offset of face f (0..2 low x,y,z; 3..5 high x,y,z) in a step, 0 if absent
    int rfcnt[3];              // cells of an x, y, z face: the product of R's other two extents
};

// ------------------------------------------------------------------ indexing
template <typename T>
__device__ __forceinline__ long long fidx(const DomDev<T>& d, int i, int j, int k) {
    return (long long)k * d.plane + (long long)j * d.pitch + i;
}

__device__ __forceinline__ int coord(int a, int i, int j, int k) { return a == 0 ? i : (a == 1 ? j : k); }

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
__device__ __forceinline__ bool in_box(const int lo[3], const int hi[3], int i, int j, int k) {
    return i >= lo[0] && i < hi[0] && j >= lo[1] && j < hi[1] && k >= lo[2] && k < hi[2];
}

template <typename T>
__device__ __forceinline__ T epsinv_at(const DomDev<T>& d, int c, int i, int j, int k) {
    if (in_box<T>(d.elo, d.ehi, i, j, k)) {
        long long q = ((long long)(k - d.elo[2]) * (d.ehi[1] - d.elo[1]) + (j - d.elo[1])) * d.exs + (i - d.exa);
        return gp(d.epsinv[c])[q];
    }
    return d.epsinv_bg;
}

template <typename T>
__device__ __forceinline__ bool in_lor(const DomDev<T>& d, int i, int j, int k) {
    return d.has_lor && in_box<T>(d.llo, d.lhi, i, j, k);
}

template <typename T>
__device__ __forceinline__ long long lidx(const DomDev<T>& d, int i, int j, int k) {
    return ((long long)(k - d.llo[2]) * (d.lhi[1] - d.llo[1]) + (j - d.llo[1])) * (d.lhi[0] - d.llo[0]) +
           (i - d.llo[0]);
}

// PEC: E_c is held at zero where the index along c+1 or c+2 is 0
__device__ __forceinline__ bool e_masked(int c, int i, int j, int k) {
    return coord((c + 1) % 3, i, j, k) == 0 || coord((c + 2) % 3, i, j, k) == 0;
}

// the same with the domain's periodic axes, which have no wall (forward paths)
template <typename T>
__device__ __forceinline__ bool e_masked_d(const DomDev<T>& d, int c, int i, int j, int k) {
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    return (coord(a1, i, j, k) == 0 && !d.per[a1]) || (coord(a2, i, j, k) == 0 && !d.per[a2]);
}

// a field one node back (x[a] - 1) / forward (x[a] + 1) along axis a = 0, 1
// from flat index f: the ghost zero past a wall, across a periodic seam the
// node at the other end times the real Bloch factor
template <typename T>
__device__ __forceinline__ T nb_back(const DomDev<T>& d, const FDTD_GLOBAL T* F, long long f, int a, int x) {
    const long long s = a == 0 ? 1 : (long long)d.pitch;
    if (x > 0) return F[f - s];
    return d.per[a] ? d.bsign[a] * F[f + (long long)(d.n[a] - 1) * s] : T(0);
}

template <typename T>
__device__ __forceinline__ T nb_fwd(const DomDev<T>& d, const FDTD_GLOBAL T* F, long long f, int a, int x) {
    const long long s = a == 0 ? 1 : (long long)d.pitch;
    if (x + 1 < d.n[a]) return F[f + s];
    return d.per[a] ? d.bsign[a] * F[f - (long long)(d.n[a] - 1) * s] : T(0);
}

// ---------------------------------------------------------- forward pieces
// Stretched difference of one curl term: D is the raw difference along axis
// a at node (i,j,k), r the slab slot, toff 0 (E side) or 3 (H side) in the
// tables.  psi_new = b psi + c D, returns D / kappa + psi_new; the owner
// stores psi_new into set ws.
template <typename T>
__device__ __forceinline__ T stretch(const DomDev<T>& d, T* const (&psi)[3][2][2], long long stride, int rs, int ws,
                                     bool own, int a, int r, int toff, int i, int j, int k, T D) {
    int x = coord(a, i, j, k);
    int s = slab_side(d, a, x);
    if (s < 0) return D;
    const FDTD_GLOBAL T* tb = gp(d.tab[a]);
    int n = d.n[a];
    T b = tb[(toff + 0) * n + x], c = tb[(toff + 1) * n + x], ki = tb[(toff + 2) * n + x];
    FDTD_GLOBAL T* base = gp(psi[a][s][r]) + pidx(d, a, s, i, j, k);
    T pn = fma(b, base[rs * stride], c * D);
    if (own) base[ws * stride] = pn;
    return fma(ki, D, pn);
}

// E^{n+1}_c at an unmasked or masked node (i,j,k) from H^{n+1/2} of set rs:
// h0 = H_{c+2} at the node and h0m one step back along a0 = c+1; h1 = H_{c+1}
// and h1m back along a1 = c+2.  The owner writes the absorber memories and
// the Lorentz history into set ws; other callers only recompute the value.
// e_update_v takes E^n_c and eps^-1 at the node from the caller (which may
// have fetched them ahead); e_update loads them itself.
template <typename T>
__device__ __forceinline__ T e_update_v(const DomDev<T>& d, int c, int i, int j, int k, long long f, T h0, T h0m,
                                        T h1, T h1m, T e, T einv, int rs, int ws, bool own, int t) {
    const bool lorc = in_lor(d, i, j, k);
    const long long fs = d.fs;
    if (e_masked_d(d, c, i, j, k)) {
        if (own && lorc) {
            long long q = lidx(d, i, j, k) + ws * fs;
            gp(d.lor[0][c])[q] = T(0);
            for (int p = 0; p < d.npole; ++p) {
                gp(d.lor[1][c])[q + p * d.lbox] = T(0);
                gp(d.lor[2][c])[q + p * d.lbox] = T(0);
            }
        }
        return T(0);
    }
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch(d, d.psiE, fs, rs, ws, own, a0, 0, 0, i, j, k, h0 - h0m);
    T D1 = stretch(d, d.psiE, fs, rs, ws, own, a1, 1, 0, i, j, k, h1 - h1m);
    T curl = D0 - D1;
    T en;
    long long q = 0;
    T eold = 0;
    if (lorc) {
        // poles' currents add: num = eps E^n + lgs/4 E^{n-1} + S curl - sum_p ((1+al_p) W_p^n + xi_p W_p^{n-1})/2
        q = lidx(d, i, j, k);
        eold = gp(d.lor[0][c])[q + rs * fs];
        T einf = T(1) / einv;
        T invden = T(1) / (einf + T(0.25) * d.lgs);
        T num = fma(einf, e, T(0.25) * d.lgs * eold);
        num = fma(d.S, curl, num);
        for (int p = 0; p < d.npole; ++p) {
            const long long o = q + p * d.lbox + rs * fs;
            const T w = gp(d.lor[1][c])[o], wold = gp(d.lor[2][c])[o];
            num -= T(0.5) * fma(T(1) + d.lal[p], w, d.lxi[p] * wold);
        }
        en = num * invden;
    } else {
        en = fma(d.S * einv, curl, e);
    }
    for (int s = 0; s < d.nsrc; ++s) {
        const SrcDev<T>& sr = d.src[s];
        if (sr.comp == c && t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j))) en += gp(sr.wave)[t];
    }
    if (own && lorc) {
        for (int p = 0; p < d.npole; ++p) {   // each pole's roll reads its own entries before writing them
            const long long o = q + p * d.lbox;
            const T w = gp(d.lor[1][c])[o + rs * fs], wold = gp(d.lor[2][c])[o + rs * fs];
            T wn = fma(d.lal[p], w, d.lxi[p] * wold);
            wn = fma(T(0.5) * d.lg[p], en - eold, wn);
            gp(d.lor[1][c])[o + ws * fs] = wn;
            gp(d.lor[2][c])[o + ws * fs] = w;
        }
        gp(d.lor[0][c])[q + ws * fs] = e;
    }
    return en;
}

template <typename T>
__device__ __forceinline__ T e_update(const DomDev<T>& d, int c, int i, int j, int k, long long f, T h0, T h0m,
                                      T h1, T h1m, int rs, int ws, bool own, int t) {
    T e = e_masked_d(d, c, i, j, k) ? T(0) : gp(d.E[c])[f + rs * d.fs];
    T einv = e_masked_d(d, c, i, j, k) ? T(0) : epsinv_at(d, c, i, j, k);
    return e_update_v(d, c, i, j, k, f, h0, h0m, h1, h1m, e, einv, rs, ws, own, t);
}

// Bulk E update (no absorber, no mask, no Lorentz, no source at the node).
template <typename T>
__device__ __forceinline__ T e_bulk(const DomDev<T>& d, int c, int i, int j, int k, long long f, T h0, T h0m, T h1,
                                    T h1m, int rs) {
    T curl = (h0 - h0m) - (h1 - h1m);
    return fma(d.S * epsinv_at(d, c, i, j, k), curl, gp(d.E[c])[f + rs * d.fs]);
}

// H^{n+3/2}_c at node (i,j,k) from E^{n+1}: e0p/e0 = E_{c+2} one step forward
// along a0 = c+1 and at the node; e1p/e1 = E_{c+1} forward along a1 = c+2.
// hold is H^{n+1/2}_c at the node.
template <typename T>
__device__ __forceinline__ T h_update(const DomDev<T>& d, int c, int i, int j, int k, T hold, T e0p, T e0, T e1p,
                                      T e1, int rs, int ws, bool own) {
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch(d, d.psiH, d.fs, rs, ws, own, a0, 0, 3, i, j, k, e0p - e0);
    T D1 = stretch(d, d.psiH, d.fs, rs, ws, own, a1, 1, 3, i, j, k, e1p - e1);
    return fma(-d.S, D0 - D1, hold);
}

template <typename T>
__device__ __forceinline__ T h_bulk(const DomDev<T>& d, T hold, T e0p, T e0, T e1p, T e1) {
    return fma(-d.S, (e0p - e0) - (e1p - e1), hold);
}

// Stretched backward-difference curl of the forward H (set rs) at an E node,
// read only (the gradient needs it from u^n without touching the state).
template <typename T>
__device__ __forceinline__ T curl_minus_ro(const DomDev<T>& d, int c, int i, int j, int k, T h0, T h0m, T h1, T h1m,
                                           int rs) {
    const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
    T D0 = stretch(d, d.psiE, d.fs, rs, rs, false, a0, 0, 0, i, j, k, h0 - h0m);
    T D1 = stretch(d, d.psiE, d.fs, rs, rs, false, a1, 1, 0, i, j, k, h1 - h1m);
    return D0 - D1;
}

// ---------------------------------------------------------- adjoint pieces
// Transposed absorber recursion (Section 3.1): from the cotangent ybar of the
// stretched derivative and the memory cotangent psibar, the cotangent of the
// raw difference is ki*ybar + c*(psibar + ybar) and the memory cotangent
// becomes b*(psibar + ybar) (stored by the owner into set ws).
template <typename T>
__device__ __forceinline__ T stretch_T(const DomDev<T>& d, T* const (&psi)[3][2][2], int rs, int ws, bool own, int a,
                                       int r, int toff, int i, int j, int k, T ybar) {
    int x = coord(a, i, j, k);
    int s = slab_side(d, a, x);
    if (s < 0) return ybar;
    const FDTD_GLOBAL T* tb = gp(d.tab[a]);
    int n = d.n[a];
    T b = tb[(toff + 0) * n + x], c = tb[(toff + 1) * n + x], ki = tb[(toff + 2) * n + x];
    FDTD_GLOBAL T* base = gp(psi[a][s][r]) + pidx(d, a, s, i, j, k);
    T mem = base[rs * d.as] + ybar;
    if (own) base[ws * d.as] = b * mem;
    return fma(ki, ybar, c * mem);
}

// Cotangent of the raw forward difference d+_a E of the H_h update term
// (a, sign, r) at H node (i,j,k): ybar = -S sign Hbar_h.
template <typename T>
__device__ __forceinline__ T hT_dbar(const DomDev<T>& d, int a, int r, T sgn, int i, int j, int k, T hbar, int rs,
                                     int ws, bool own) {
    return stretch_T(d, d.psiHa, rs, ws, own, a, r, 3, i, j, k, -d.S * sgn * hbar);
}

// E-update transpose at E node c.  From etot (cotangent of E^{n+1} after the
// H transpose) returns the cotangent of E^{n+1} before the source (epre) and
// the coefficient of the curl (eps^-1 or 1/den).  The owner applies the
// Lorentz history transpose into set ws and gets the new cotangent of E^n.
template <typename T>
struct AdjE {
    T epre, coef, en;
};

template <typename T>
__device__ __forceinline__ AdjE<T> et_node(const DomDev<T>& d, int c, int i, int j, int k, T etot, int rs, int ws,
                                           bool own) {
    AdjE<T> r;
    r.epre = T(0);
    r.coef = T(0);
    r.en = T(0);
    const long long as = d.as;
    if (e_masked(c, i, j, k)) {
        if (own && in_lor(d, i, j, k)) {
            long long q = lidx(d, i, j, k) + ws * as;
            gp(d.lora[0][c])[q] = T(0);
            for (int p = 0; p < d.npole; ++p) {
                gp(d.lora[1][c])[q + p * d.lbox] = T(0);
                gp(d.lora[2][c])[q + p * d.lbox] = T(0);
            }
        }
        return r;
    }
    T einv = epsinv_at(d, c, i, j, k);
    if (in_lor(d, i, j, k)) {
        long long q = lidx(d, i, j, k);
        T einf = T(1) / einv;
        T invden = T(1) / (einf + T(0.25) * d.lgs);
        T ep = etot;
        for (int p = 0; p < d.npole; ++p)        // each pole's W^{n+1} roll feeds E^{n+1}
            ep = fma(T(0.5) * d.lg[p], gp(d.lora[1][c])[q + p * d.lbox + rs * as], ep);
        r.epre = ep;
        r.coef = invden;
        if (own) {
            T eob = gp(d.lora[0][c])[q + rs * as];
            T s = ep * invden;
            r.en = fma(einf, s, eob);
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
template <typename T>
__device__ __forceinline__ T et_dbar(const DomDev<T>& d, int a, int r, T sgn, int i, int j, int k, T epre, T coef,
                                     int rs, int ws, bool own) {
    return stretch_T(d, d.psiEa, rs, ws, own, a, r, 0, i, j, k, d.S * coef * sgn * epre);
}

// dJ/deps_c contribution of one E node from the forward state u^n (set fsr):
// -S eps^-2 Ebar_pre curl (dielectric), Ebar_pre (E^n - E^{n+1}_pre)/den (Lorentz).
template <typename T>
__device__ __forceinline__ double grad_term(const DomDev<T>& d, int c, int i, int j, int k, long long f, T epre,
                                            T h0, T h0m, T h1, T h1m, int fsr) {
    T curl = curl_minus_ro(d, c, i, j, k, h0, h0m, h1, h1m, fsr);
    T einv = epsinv_at(d, c, i, j, k);
    if (in_lor(d, i, j, k)) {
        long long q = lidx(d, i, j, k) + fsr * d.fs;
        T e = gp(d.E[c])[f + fsr * d.fs];
        T eold = gp(d.lor[0][c])[q];
        T einf = T(1) / einv;
        T invden = T(1) / (einf + T(0.25) * d.lgs);
        T num = fma(einf, e, T(0.25) * d.lgs * eold);
        num = fma(d.S, curl, num);
        for (int p = 0; p < d.npole; ++p) {
            const T w = gp(d.lor[1][c])[q + p * d.lbox], wold = gp(d.lor[2][c])[q + p * d.lbox];
            num -= T(0.5) * fma(T(1) + d.lal[p], w, d.lxi[p] * wold);
        }
        T epre_f = num * invden;
        return (double)epre * (double)((e - epre_f) * invden);
    }
    return -(double)epre * (double)(d.S * einv * einv * curl);
}

template <typename T>
__device__ __forceinline__ bool in_gbox(const DomDev<T>& d, int i, int j, int k) {
    return d.grad && in_box<T>(d.glo, d.ghi, i, j, k);
}

template <typename T>
__device__ __forceinline__ void grad_store(const DomDev<T>& d, int i, int j, int k, const double g[3]) {
    long long q = ((long long)(k - d.glo[2]) * (d.ghi[1] - d.glo[1]) + (j - d.glo[1])) * (d.ghi[0] - d.glo[0]) +
                  (i - d.glo[0]);
    if (d.eps_diag) {
        gp(d.gacc[0])[q] += g[0];
        gp(d.gacc[1])[q] += g[1];
        gp(d.gacc[2])[q] += g[2];
    } else {
        gp(d.gacc[0])[q] += (g[0] + g[1]) + g[2];
    }
}

}  // namespace fdtd
