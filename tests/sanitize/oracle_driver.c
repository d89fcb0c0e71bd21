/*
 * Host memory-safety driver for the FP64 oracle (test infrastructure): it
 * compiles the oracle source into one program with the address and
 * undefined-behaviour sanitizers and runs forward and adjoint steps, with
 * gradients, on small ragged domains covering every branch: absorbing faces
 * on all sides, a dispersive box of two poles, Bloch-periodic x and y with a
 * dispersive box on the seam, and symmetric tensor media.  The values are
 * arbitrary (stable enough to stay finite); what is checked is that every
 * access stays inside its array and the results are finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/fdtd_oracle.c"

static double *zalloc(size_t n) {
    double *p = (double *)calloc(n ? n : 1, sizeof(double));
    if (!p) {
        fprintf(stderr, "allocation failed\n");
        exit(2);
    }
    return p;
}

static double urand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

typedef struct {
    double *arrays[128];
    int n;
} pool;

static double *take(pool *pl, size_t n) {
    if (pl->n >= 128) {
        fprintf(stderr, "driver pool full\n");
        exit(2);
    }
    double *p = zalloc(n);
    pl->arrays[pl->n++] = p;
    return p;
}

/* kind 0: walled, absorbing faces, two-pole box; 1: periodic x, y with a box on the seam; 2: tensor media */
static int run_case(int kind) {
    const int n[3] = {7, 6, 9};
    const size_t N = (size_t)n[0] * n[1] * n[2];
    unsigned seed = 12345u + (unsigned)kind;
    pool pl = {{0}, 0};
    orc_params P;
    memset(&P, 0, sizeof P);
    for (int a = 0; a < 3; ++a) P.n[a] = n[a];
    P.S = 0.99 / sqrt(3.0);
    unsigned char *slab[3];
    for (int a = 0; a < 3; ++a) {
        double *t = take(&pl, 6 * (size_t)n[a]);
        slab[a] = (unsigned char *)calloc((size_t)n[a], 1);
        const int per = kind == 1 && a < 2;
        for (int i = 0; i < n[a]; ++i) {
            const int in = !per && (i < 2 || i >= n[a] - 2);
            slab[a][i] = (unsigned char)in;
            t[0 * n[a] + i] = in ? 0.7 : 1.0;   /* b */
            t[1 * n[a] + i] = in ? -0.1 : 0.0;  /* c */
            t[2 * n[a] + i] = in ? 0.8 : 1.0;   /* 1/kappa */
            t[3 * n[a] + i] = in ? 0.7 : 1.0;
            t[4 * n[a] + i] = in ? -0.1 : 0.0;
            t[5 * n[a] + i] = in ? 0.8 : 1.0;
        }
        P.bE[a] = t;
        P.cE[a] = t + n[a];
        P.kiE[a] = t + 2 * n[a];
        P.bH[a] = t + 3 * n[a];
        P.cH[a] = t + 4 * n[a];
        P.kiH[a] = t + 5 * n[a];
        P.slab[a] = slab[a];
        P.per[a] = per;
        P.bsign[a] = a == 0 ? -1.0 : 1.0;
    }
    for (int c = 0; c < 3; ++c) {
        double *e = take(&pl, N);
        for (size_t p = 0; p < N; ++p) e[p] = 1.0 + 2.0 * urand(&seed);
        P.eps[c] = e;
    }
    unsigned char *lor = NULL;
    if (kind < 2) {
        lor = (unsigned char *)calloc(N, 1);
        for (int k = 2; k < 6; ++k)
            for (int j = 1; j < 4; ++j)
                for (int i = 0; i < (kind == 1 ? 3 : 5); ++i) lor[IDX(&P, i, j, k)] = 1;
        P.lor = lor;
        P.npole = 2;
        P.pkind[0] = 0;
        P.pdeps[0] = 1.2;
        P.pwdt[0] = 0.4;
        P.pgdt[0] = 0.02;
        P.pkind[1] = 1;
        P.pwdt[1] = 0.3;
        P.pgdt[1] = 0.05;
    }
    if (kind == 2) {
        /* eps^-1 at the nodes: a diagonal in (0.25, 0.9) and off-diagonal entries of 0.02 */
        for (int q = 0; q < 6; ++q) {
            double *t = take(&pl, N);
            for (size_t p = 0; p < N; ++p) t[p] = q < 3 ? 0.25 + 0.65 * urand(&seed) : 0.02;
            P.einvT[q] = t;
        }
        P.einv_bg = 1.0;
    }
    orc_state U, A;
    memset(&U, 0, sizeof U);
    memset(&A, 0, sizeof A);
    orc_state *st[2] = {&U, &A};
    for (int s = 0; s < 2; ++s) {
        for (int q = 0; q < 6; ++q) st[s]->F[q] = take(&pl, N);
        for (int c = 0; c < 3; ++c) {
            for (int a = 0; a < 3; ++a) {
                st[s]->psiE[c][a] = take(&pl, N);
                st[s]->psiH[c][a] = take(&pl, N);
            }
        }
    }
    double *hist[2][3][5];   /* Eold, W0, W1, Wold0, Wold1 per component (shared size N) */
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 3; ++c)
            for (int h = 0; h < 5; ++h) {
                hist[s][c][h] = zalloc(N);
            }
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 3; ++c) {
            st[s]->Eold[c] = hist[s][c][0];
            st[s]->W[c][0] = hist[s][c][1];
            st[s]->W[c][1] = hist[s][c][2];
            st[s]->Wold[c][0] = hist[s][c][3];
            st[s]->Wold[c][1] = hist[s][c][4];
        }
    double *work = zalloc(7 * N);
    const int nsrc = 2;
    const int src_comp[2] = {0, 2};
    const long long src_idx[2] = {(long long)IDX(&P, 3, 3, 4), (long long)IDX(&P, 0, 0, 0)};
    double amp[2];
    for (int t = 0; t < 6; ++t) {
        amp[0] = sin(0.3 * t);
        amp[1] = cos(0.2 * t);
        orc_step(&P, &U, nsrc, src_comp, src_idx, amp, work);
    }
    for (int q = 0; q < 6; ++q)
        for (size_t p = 0; p < N; ++p) A.F[q][p] = urand(&seed) - 0.5;
    double *g[6];
    const int ng = kind == 2 ? 6 : 3;
    for (int q = 0; q < ng; ++q) g[q] = take(&pl, N);
    for (int t = 0; t < 6; ++t) orc_adjoint_step(&P, &A, &U, g, work);
    int bad = 0;
    for (int q = 0; q < 6; ++q)
        for (size_t p = 0; p < N; ++p)
            if (!isfinite(U.F[q][p]) || !isfinite(A.F[q][p])) bad = 1;
    for (int q = 0; q < ng; ++q)
        for (size_t p = 0; p < N; ++p)
            if (!isfinite(g[q][p])) bad = 1;
    for (int q = 0; q < pl.n; ++q) free(pl.arrays[q]);
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 3; ++c)
            for (int h = 0; h < 5; ++h) free(hist[s][c][h]);
    for (int a = 0; a < 3; ++a) free(slab[a]);
    free(lor);
    free(work);
    printf("case %d: %s\n", kind, bad ? "non-finite values" : "ok");
    return bad;
}

int main(void) {
    int bad = 0;
    for (int kind = 0; kind < 3; ++kind) bad |= run_case(kind);
    return bad;
}
