/*
 * fdtd_oracle.c -- plain FP64 CPU oracle of the differentiable FDTD step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source with the HIP path.
 *
 * It is written for a reader holding the paper (TorchFDTD, arXiv 2609.30039):
 *   - Yee leapfrog, Eq. (1) of Section 2.1: E += S eps^-1 C^-(H) + s,
 *     then H -= S C^+(E).  Unit mesh, c = 1, so dt = S.
 *   - Convolutional PML (Section 2.2): a psi memory for each tangential
 *     difference taken inside an absorbing slab; forward form psi <- b psi + c D,
 *     Dt = D / kappa + psi (the form whose transpose Section 3.1 prints).
 *   - PEC faces (Section 2.2): tangential E held at zero on the low boundary
 *     node; the high boundary node is not stored (ghost zero).
 *   - Dispersive cells with up to 16 Lorentz or Drude poles by the
 *     trapezoidal auxiliary differential equation (Section 2.3): Ampere at
 *     n+1/2 with the trapezoidal average of the polarisation currents, each
 *     pole's ODE by central differences at n; the poles' currents add.  A
 *     Drude pole is the Lorentz recursion with omega_0 -> 0 and
 *     delta_eps omega_0^2 -> omega_p^2.
 *   - Symmetric tensor media (Section 2.3): eps at the grid nodes, inverted
 *     there, and applied to the curl through the node assembly
 *     (1/8) sum over the eight octants of R^T eps^-1 R (across a periodic
 *     seam the node and edges at the other end, the edges times the Bloch
 *     factor); its transpose is itself, and the gradient of a node's tensor
 *     collects, octant by octant, the outer product of the E cotangent and
 *     the curl on the octant's edges.
 *   - Discrete adjoint, Eq. (3) of Section 3.1, with the transposes of
 *     Section 3.1 (opposite-direction differences, the absorber transpose,
 *     the 2x2 dispersion transpose, eps cotangent = E cotangent x curl, and
 *     across a periodic seam the conjugate of the Bloch factor, which is the
 *     factor itself for the real factors +1 and -1).
 *
 * Arrays are [nz][ny][nx], x fastest, one full-grid array per quantity.
 * Every loop is a plain loop over the grid; OpenMP splits the outer z loop
 * only where the iterations write disjoint nodes.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n[3];                    /* cells along x, y, z (absorbing cells included) */
    double S;                    /* Courant number c dt / h */
    /* absorber tables along each axis a, indexed by the node index along a.
       E-update derivatives are sampled at integer positions, H-update
       derivatives at half-integer positions. slab[a][i] = 1 inside a face. */
    const double *bE[3], *cE[3], *kiE[3];
    const double *bH[3], *cH[3], *kiH[3];
    const unsigned char *slab[3];
    const double *eps[3];        /* permittivity at each E node, per component */
    const unsigned char *lor;    /* 1 where the cell is a dispersive cell, or NULL */
    int npole;                   /* poles of the dispersive cells, 1..ORC_MAXP */
    int pkind[16];               /* 0 Lorentz, 1 Drude */
    double pdeps[16];            /* Lorentz: delta eps (Drude: unused) */
    double pwdt[16];             /* Lorentz: omega_0 dt; Drude: omega_p dt */
    double pgdt[16];             /* gamma dt */
    int per[3];                  /* 1: the axis is periodic (Bloch, Section 2.2): no PEC wall, the
                                    neighbour past the last node is the first one times bsign */
    double bsign[3];             /* real Bloch factor exp(i k L) = +1 or -1 of a periodic axis */
    /* symmetric tensor media (Section 2.3): eps^-1 at the grid nodes, components
       xx, yy, zz, xy, xz, yz, one full-grid array each (node (i,j,k) is the corner
       where the edges Ex, Ey, Ez of index (i,j,k) start); NULL: eps per E node */
    const double *einvT[6];
    double einv_bg;              /* eps^-1 of the nodes past the arrays' high end */
} orc_params;

#define ORC_MAXP 16

typedef struct {
    double *F[6];                /* Ex Ey Ez Hx Hy Hz */
    double *psiE[3][3];          /* [E component][derivative axis], diagonal unused */
    double *psiH[3][3];          /* [H component][derivative axis] */
    double *Eold[3];             /* dispersive history: E^{n-1} */
    double *W[3][16], *Wold[3][16];     /* per pole: W^n, W^{n-1} */
} orc_state;

#define IDX(P, i, j, k) (((size_t)(k) * (size_t)(P)->n[1] + (size_t)(j)) * (size_t)(P)->n[0] + (size_t)(i))

static size_t stride_of(const orc_params *P, int a) {
    return a == 0 ? 1 : (a == 1 ? (size_t)P->n[0] : (size_t)P->n[0] * (size_t)P->n[1]);
}

/* PEC: E component c is tangential to the low faces normal to the other two
   axes; those boundary nodes are held at zero and are not degrees of freedom.
   A periodic axis has no wall. */
static int e_masked(const orc_params *P, int c, const int x[3]) {
    int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    return (x[a1] == 0 && !P->per[a1]) || (x[a2] == 0 && !P->per[a2]);
}

/* Field value one node back / forward along axis a from node p.  Past the
   domain: zero (the wall's ghost), or on a periodic axis the node at the other
   end times the Bloch factor: F(N) = bsign F(0) and F(-1) = bsign^-1 F(N-1),
   where bsign^-1 = bsign for the real factors +1 and -1. */
static double back(const orc_params *P, const double *F, const int x[3], size_t p, int a) {
    size_t s = stride_of(P, a);
    if (x[a] > 0) return F[p - s];
    return P->per[a] ? P->bsign[a] * F[p + (size_t)(P->n[a] - 1) * s] : 0.0;
}

static double fwd(const orc_params *P, const double *F, const int x[3], size_t p, int a) {
    size_t s = stride_of(P, a);
    if (x[a] < P->n[a] - 1) return F[p + s];
    return P->per[a] ? P->bsign[a] * F[p - (size_t)(P->n[a] - 1) * s] : 0.0;
}

static int is_lorentz(const orc_params *P, size_t p) { return P->lor && P->lor[p]; }

/* Recursion constants of pole p of the trapezoidal ADE with W = dt J:
   W^{n+1} = al W^n + xi W^{n-1} + (g/2)(E^{n+1} - E^{n-1}).
   Lorentz: al = (2 - (w0 dt)^2)/q, g = deps (w0 dt)^2/q; Drude: al = 2/q,
   g = (wp dt)^2/q; both xi = (gamma dt/2 - 1)/q, q = 1 + gamma dt/2. */
static void pole_consts(const orc_params *P, int p, double *al, double *xi, double *g) {
    double q = 1.0 + 0.5 * P->pgdt[p];
    double w2 = P->pwdt[p] * P->pwdt[p];
    *al = P->pkind[p] ? 2.0 / q : (2.0 - w2) / q;
    *xi = (0.5 * P->pgdt[p] - 1.0) / q;
    *g = P->pkind[p] ? w2 / q : P->pdeps[p] * w2 / q;
}

/* sum of the poles' g: the E^{n-1} weight and the denominator eps + gsum/4 */
static double pole_gsum(const orc_params *P) {
    double s = 0.0;
    for (int q = 0; q < P->npole; ++q) {
        double al, xi, g;
        pole_consts(P, q, &al, &xi, &g);
        s += g;
    }
    return s;
}

/* Stretched backward-difference curl of H at E node p (component c):
   (C^- H)_c = d-_{c+1} H_{c+2} - d-_{c+2} H_{c+1}.
   With write_psi the updated absorber memories are stored (forward step);
   without, they are only used to form the value (gradient recomputation). */
static double curl_minus(const orc_params *P, const orc_state *U, int c, const int x[3], size_t p,
                         int write_psi) {
    double acc = 0.0;
    for (int t = 0; t < 2; ++t) {
        int a = (c + 1 + t) % 3;
        int h = t == 0 ? (c + 2) % 3 : (c + 1) % 3;
        double sgn = t == 0 ? 1.0 : -1.0;
        const double *H = U->F[3 + h];
        double D = H[p] - back(P, H, x, p, a);
        double Dt = D;
        if (P->slab[a][x[a]]) {
            double *psi = U->psiE[c][a];
            double pn = P->bE[a][x[a]] * psi[p] + P->cE[a][x[a]] * D;
            if (write_psi) psi[p] = pn;
            Dt = P->kiE[a][x[a]] * D + pn;
        }
        acc += sgn * Dt;
    }
    return acc;
}

/* Stretched forward-difference curl of E at H node p (component c):
   (C^+ E)_c = d+_{c+1} E_{c+2} - d+_{c+2} E_{c+1}; updates the H memories. */
static double curl_plus(const orc_params *P, orc_state *U, int c, const int x[3], size_t p) {
    double acc = 0.0;
    for (int t = 0; t < 2; ++t) {
        int a = (c + 1 + t) % 3;
        int e = t == 0 ? (c + 2) % 3 : (c + 1) % 3;
        double sgn = t == 0 ? 1.0 : -1.0;
        const double *E = U->F[e];
        double D = fwd(P, E, x, p, a) - E[p];
        double Dt = D;
        if (P->slab[a][x[a]]) {
            double *psi = U->psiH[c][a];
            psi[p] = P->bH[a][x[a]] * psi[p] + P->cH[a][x[a]] * D;
            Dt = P->kiH[a][x[a]] * D + psi[p];
        }
        acc += sgn * Dt;
    }
    return acc;
}

/* E^{n+1} before the source, from u^n, at one unmasked node. */
static double e_pre(const orc_params *P, const orc_state *U, int c, size_t p, double curl) {
    double ep = P->eps[c][p];
    if (is_lorentz(P, p)) {
        double gsum = pole_gsum(P);
        double den = ep + 0.25 * gsum;
        double num = ep * U->F[c][p] + 0.25 * gsum * U->Eold[c][p] + P->S * curl;
        for (int q = 0; q < P->npole; ++q) {
            double al, xi, g;
            pole_consts(P, q, &al, &xi, &g);
            num -= 0.5 * ((1.0 + al) * U->W[c][q][p] + xi * U->Wold[c][q][p]);
        }
        return num / den;
    }
    return U->F[c][p] + P->S * curl / ep;
}

/*
 * One forward step u^n -> u^{n+1}, in the order
 *   1. E (or Lorentz-ADE) update with the absorber memories, PEC nodes kept,
 *   2. soft electric sources s^{n+1} (PEC nodes skipped),
 *   3. Lorentz history roll with the post-source E^{n+1},
 *   4. H update with its absorber memories.
 * src_*: the increments of this step.  work: three full-grid scratch arrays.
 */
/* eps^-1 component (a, b) at node v.  Nodes past the arrays' high end take
   the background, or on a periodic axis are the node at the other end (the
   medium repeats; the Bloch factor multiplies fields, not materials). */
static double node_einv(const orc_params *P, const int v[3], int a, int b) {
    int w[3] = {v[0], v[1], v[2]};
    for (int q = 0; q < 3; ++q)
        if (w[q] >= P->n[q]) {
            if (!P->per[q]) return a == b ? P->einv_bg : 0.0;
            w[q] -= P->n[q];
        }
    static const int comp[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    return P->einvT[comp[a][b]][IDX(P, w[0], w[1], w[2])];
}

/* value of the E-edge array Cc of component b at the edge starting at node v:
   zero past a wall; across a periodic seam the edge at the other end times
   the Bloch factor (F(N) = bsign F(0), F(-1) = bsign F(N-1) for the real
   factors).  The caller zeroes masked edges. */
static double edge_curl(const orc_params *P, double *const Cc[3], int b, const int v[3]) {
    int w[3] = {v[0], v[1], v[2]};
    double fac = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (w[a] >= 0 && w[a] < P->n[a]) continue;
        if (!P->per[a]) return 0.0;
        w[a] += w[a] < 0 ? P->n[a] : -P->n[a];
        fac *= P->bsign[a];
    }
    return fac * Cc[b][IDX(P, w[0], w[1], w[2])];
}

/* The node-assembled tensor applied to the curl, at the E edge of component c
   starting at node x (Section 2.3, S = D^-1/2 (1/8 sum_s R_s^T eps^-1 R_s)
   D^-1/2 with D the identity on the unit mesh).  The edge belongs to its two end
   nodes; at each, the eight octants pick one x, one y and one z edge incident
   to the node, and the four octants holding this edge contribute
   eps^-1_cc c_c + eps^-1_cb c_b(octant's b edge) for b != c, each times 1/8. */
static double tensor_apply(const orc_params *P, double *const Cc[3], int c, const int x[3]) {
    double acc = 0.0;
    for (int end = 0; end < 2; ++end) {
        int v[3] = {x[0], x[1], x[2]};
        v[c] += end;
        acc += 0.5 * node_einv(P, v, c, c) * Cc[c][IDX(P, x[0], x[1], x[2])];
        for (int t = 1; t < 3; ++t) {
            int b = (c + t) % 3;
            int w[3] = {v[0], v[1], v[2]};
            double s = edge_curl(P, Cc, b, w);        /* the b edge leaving the node */
            w[b] -= 1;
            s += edge_curl(P, Cc, b, w);              /* the b edge arriving at it */
            acc += 0.25 * node_einv(P, v, c, b) * s;
        }
    }
    return acc;
}

void orc_step(const orc_params *P, orc_state *U, int nsrc, const int *src_comp, const long long *src_idx,
              const double *src_amp, double *work) {
    const int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const size_t N = (size_t)nx * ny * nz;
    if (P->einvT[0]) {
        /* tensor media: the stretched curl of every E edge first (absorber
           memories updated, masked edges zero), then E += S (assembled eps^-1) curl */
        double *Cc[3] = {work, work + N, work + 2 * N};
        for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        Cc[c][p] = e_masked(P, c, x) ? 0.0 : curl_minus(P, U, c, x, p, 1);
                    }
        }
        for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        if (e_masked(P, c, x)) continue;
                        U->F[c][IDX(P, i, j, k)] += P->S * tensor_apply(P, Cc, c, x);
                    }
        }
    } else
    for (int c = 0; c < 3; ++c) {
        double *En = work + (size_t)c * N;      /* E^n of Lorentz nodes, for the roll */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int x[3] = {i, j, k};
                    if (e_masked(P, c, x)) continue;
                    size_t p = IDX(P, i, j, k);
                    double curl = curl_minus(P, U, c, x, p, 1);
                    double en1 = e_pre(P, U, c, p, curl);
                    En[p] = U->F[c][p];
                    U->F[c][p] = en1;
                }
    }
    for (int s = 0; s < nsrc; ++s) {
        size_t p = (size_t)src_idx[s];
        int c = src_comp[s];
        int x[3] = {(int)(p % nx), (int)((p / nx) % ny), (int)(p / ((size_t)nx * ny))};
        if (e_masked(P, c, x)) continue;
        U->F[c][p] += src_amp[s];
    }
    if (P->lor) {
        for (int c = 0; c < 3; ++c) {
            const double *En = work + (size_t)c * N;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        if (!P->lor[p] || e_masked(P, c, x)) continue;
                        for (int q = 0; q < P->npole; ++q) {
                            double al, xi, g;
                            pole_consts(P, q, &al, &xi, &g);
                            double wn1 = al * U->W[c][q][p] + xi * U->Wold[c][q][p]
                                         + 0.5 * g * (U->F[c][p] - U->Eold[c][p]);
                            U->Wold[c][q][p] = U->W[c][q][p];
                            U->W[c][q][p] = wn1;
                        }
                        U->Eold[c][p] = En[p];
                    }
        }
    }
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int x[3] = {i, j, k};
                    size_t p = IDX(P, i, j, k);
                    U->F[3 + c][p] -= P->S * curl_plus(P, U, c, x, p);
                }
    }
}

/* Absorber transpose (Section 3.1): given the cotangent ybar of the stretched
   derivative and the cotangent of the stored memory, return the cotangent of
   the raw difference and leave the cotangent of the previous memory. */
static double cpml_T(double ybar, double *psibar, double b, double c, double ki) {
    double mem = *psibar + ybar;
    double Dbar = ki * ybar + c * mem;
    *psibar = b * mem;
    return Dbar;
}

/*
 * One adjoint step ubar^{n+1} -> (dF_n/du)^T ubar^{n+1}, in place in A, and
 * accumulation of the permittivity gradient dJ/deps_c into g[c] (when g is
 * non-null) from the forward state U = u^n.  The seeds dJ/du^n are added by
 * the caller.  The order is the reverse of orc_step: H transpose, Lorentz
 * history transpose, E transpose.  Tensor media: g holds six arrays, dJ/dp
 * for the stored entries xx yy zz xy xz yz of eps^-1 at the nodes (an
 * off-diagonal entry is one parameter for both of its matrix entries).
 * work: four full-grid scratch arrays, seven for tensor media.
 */
void orc_adjoint_step(const orc_params *P, orc_state *A, const orc_state *U, double **g, double *work) {
    const int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const size_t N = (size_t)nx * ny * nz;
    double *Dbar = work;
    double *Epb[3] = {work + N, work + 2 * N, work + 3 * N};   /* cotangent of E^{n+1} before the source */

    /* ---- H transpose: H_c -= S * sgn * Dt(d+_a E_e) ---- */
    for (int c = 0; c < 3; ++c)
        for (int t = 0; t < 2; ++t) {
            int a = (c + 1 + t) % 3;
            int e = t == 0 ? (c + 2) % 3 : (c + 1) % 3;
            double sgn = t == 0 ? 1.0 : -1.0;
            size_t sa = stride_of(P, a);
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        double ybar = -P->S * sgn * A->F[3 + c][p];
                        if (P->slab[a][x[a]])
                            Dbar[p] = cpml_T(ybar, &A->psiH[c][a][p], P->bH[a][x[a]], P->cH[a][x[a]],
                                             P->kiH[a][x[a]]);
                        else
                            Dbar[p] = ybar;
                    }
            /* D[i] = E[i+1] - E[i] (E beyond the grid is zero, or on a periodic
               axis E[N] = bsign E[0])  =>  Ebar[i] += Dbar[i-1] - Dbar[i], and
               Ebar[0] takes bsign Dbar[N-1] across the seam (the transposed
               factor: the conjugate, equal to bsign for the real factors) */
            const double seam = P->per[a] ? P->bsign[a] : 0.0;
            const size_t wrap = (size_t)(P->n[a] - 1) * sa;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        A->F[e][p] += (x[a] > 0 ? Dbar[p - sa] : seam * Dbar[p + wrap]) - Dbar[p];
                    }
        }

    /* ---- dispersive history and E-update transposes, pointwise ---- */
    const double gg = P->lor ? pole_gsum(P) : 0.0;
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    int x[3] = {i, j, k};
                    size_t p = IDX(P, i, j, k);
                    if (e_masked(P, c, x)) {
                        A->F[c][p] = 0.0;
                        Epb[c][p] = 0.0;
                        continue;
                    }
                    if (is_lorentz(P, p)) {
                        double ep = P->eps[c][p];
                        double den = ep + 0.25 * gg;
                        /* roll of each pole q: W_q^{n+1} = al_q W_q^n + xi_q W_q^{n-1}
                           + g_q/2 (E^{n+1} - E^{n-1}), Wold_q <- W_q^n; Eold <- E^n */
                        double Et = A->F[c][p];                       /* cotangent of E^{n+1} */
                        double Enm1 = 0.0;                            /* cotangent of E^{n-1} */
                        double Wn[ORC_MAXP], Wnm1[ORC_MAXP];           /* cotangents of W_q^n, W_q^{n-1} */
                        for (int q = 0; q < P->npole; ++q) {
                            double al, xi, g;
                            pole_consts(P, q, &al, &xi, &g);
                            double Wb = A->W[c][q][p];
                            Et += 0.5 * g * Wb;
                            Enm1 += -0.5 * g * Wb;
                            Wn[q] = al * Wb + A->Wold[c][q][p];
                            Wnm1[q] = xi * Wb;
                        }
                        double En = A->Eold[c][p];                    /* cotangent of E^n */
                        /* E^{n+1}_pre = [eps E^n + gsum/4 E^{n-1} + S curl
                                          - sum_q ((1+al_q) W_q^n + xi_q W_q^{n-1})/2] / den */
                        double Ep = Et;
                        En += ep / den * Ep;
                        Enm1 += 0.25 * gg / den * Ep;
                        for (int q = 0; q < P->npole; ++q) {
                            double al, xi, g;
                            pole_consts(P, q, &al, &xi, &g);
                            A->W[c][q][p] = Wn[q] + -0.5 * (1.0 + al) / den * Ep;
                            A->Wold[c][q][p] = Wnm1[q] + -0.5 * xi / den * Ep;
                        }
                        Epb[c][p] = Ep;
                        A->F[c][p] = En;
                        A->Eold[c][p] = Enm1;
                    } else {
                        Epb[c][p] = A->F[c][p];   /* E^{n+1} = E^n + ... : identity on E^n */
                    }
                }
    }

    /* ---- tensor media: the node-tensor gradient, then the curl cotangent ---- */
    double *Cb[3] = {work + 4 * N, work + 5 * N, work + 6 * N};
    if (P->einvT[0]) {
        /* the stretched curl of the forward step from u^n (memories read, not
           written), zero on masked edges: the y of E += S (assembly) y */
        for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        Cb[c][p] = e_masked(P, c, x) ? 0.0 : curl_minus(P, U, c, x, p, 0);
                    }
        }
        if (g) {
            /* dJ/dp_q for the stored entry q = (a, b) of eps^-1 at node v (one
               parameter for both A_ab and A_ba): with u = R_s (S Ebar) and
               y = R_s curl the three edges of octant s,
               dJ/dA_ab = 1/8 sum_s u_a y_b; p_ab collects A_ab and A_ba */
            static const int qa[6] = {0, 1, 2, 0, 0, 1}, qb[6] = {0, 1, 2, 1, 2, 2};
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        const int v[3] = {i, j, k};
                        const size_t pv = IDX(P, i, j, k);
                        for (int s = 0; s < 8; ++s) {
                            double u[3], y[3];
                            for (int b = 0; b < 3; ++b) {
                                int w[3] = {v[0], v[1], v[2]};
                                w[b] -= (s >> b) & 1;        /* 1: the b edge arriving at v */
                                u[b] = P->S * edge_curl(P, Epb, b, w);
                                y[b] = edge_curl(P, Cb, b, w);
                            }
                            for (int q = 0; q < 6; ++q) {
                                const int a = qa[q], b = qb[q];
                                g[q][pv] += (a == b ? u[a] * y[a] : u[a] * y[b] + u[b] * y[a]) / 8.0;
                            }
                        }
                    }
        }
        /* Cbar = S (assembly) Ebar on the unmasked edges.  The assembly is its
           own transpose: each octant's R_s^T eps^-1 R_s is symmetric, and the
           masked edges (zero in Ebar, no update) drop out of rows and columns */
        for (int c = 0; c < 3; ++c) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        Cb[c][IDX(P, i, j, k)] = e_masked(P, c, x) ? 0.0 : P->S * tensor_apply(P, Epb, c, x);
                    }
        }
    }

    /* ---- gradient: dJ/deps_c accumulates dE_pre/deps_c * Ebar_pre ---- */
    if (g && !P->einvT[0]) {
        for (int c = 0; c < 3; ++c) {
            if (!g[c]) continue;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        if (e_masked(P, c, x)) continue;
                        size_t p = IDX(P, i, j, k);
                        double curl = curl_minus(P, U, c, x, p, 0);
                        double ep = P->eps[c][p];
                        if (is_lorentz(P, p)) {
                            double den = ep + 0.25 * gg;
                            double epre = e_pre(P, U, c, p, curl);
                            g[c][p] += Epb[c][p] * (U->F[c][p] - epre) / den;
                        } else {
                            g[c][p] += -Epb[c][p] * P->S * curl / (ep * ep);
                        }
                    }
        }
    }

    /* ---- E transpose: E_c += S * coef * sgn * Dt(d-_a H_h) ---- */
    for (int c = 0; c < 3; ++c)
        for (int t = 0; t < 2; ++t) {
            int a = (c + 1 + t) % 3;
            int h = t == 0 ? (c + 2) % 3 : (c + 1) % 3;
            double sgn = t == 0 ? 1.0 : -1.0;
            size_t sa = stride_of(P, a);
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        if (e_masked(P, c, x)) {
                            Dbar[p] = 0.0;
                            continue;
                        }
                        double ybar;
                        if (P->einvT[0]) {
                            ybar = sgn * Cb[c][p];
                        } else {
                            double ep = P->eps[c][p];
                            double coef = is_lorentz(P, p) ? 1.0 / (ep + 0.25 * gg) : 1.0 / ep;
                            ybar = P->S * coef * sgn * Epb[c][p];
                        }
                        if (P->slab[a][x[a]])
                            Dbar[p] = cpml_T(ybar, &A->psiE[c][a][p], P->bE[a][x[a]], P->cE[a][x[a]],
                                             P->kiE[a][x[a]]);
                        else
                            Dbar[p] = ybar;
                    }
            /* D[i] = H[i] - H[i-1] (H below the grid is zero, or on a periodic
               axis H[-1] = bsign H[N-1])  =>  Hbar[i] += Dbar[i] - Dbar[i+1],
               and Hbar[N-1] gives up bsign Dbar[0] across the seam */
            const double seam = P->per[a] ? P->bsign[a] : 0.0;
            const size_t wrap = (size_t)(P->n[a] - 1) * sa;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        int x[3] = {i, j, k};
                        size_t p = IDX(P, i, j, k);
                        A->F[3 + h][p] += Dbar[p] - (x[a] < P->n[a] - 1 ? Dbar[p + sa] : seam * Dbar[p - wrap]);
                    }
        }
}
