/*
 * oracle.c -- plain, slow, FP64 CPU reference of the spin-aware NEP potential
 * and of the coupled spin-lattice step.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code with the HIP library.
 *
 * What it computes (paper: "Extreme-Scale Atomistic Simulation of
 * Real-Temperature Magnetic Skyrmion Dynamics by Coupled Spin-Lattice
 * Modeling"):
 *   - the unified energy surface E(R,S) as a sum of per-atom energies of a
 *     local descriptor (Sec. 5.2 "Unified spin-lattice execution"), whose
 *     channels are the structural radial/angular NEP terms plus the magnetic
 *     onsite, pairwise (exchange, DMI, anisotropic exchange, single-ion) and
 *     spin-weighted angular groups (Sec. 5.1 "A spin-aware local descriptor
 *     pipeline", "Implementation-oriented descriptor organization");
 *   - Chebyshev radial functions built by the recurrence T_{k+1}=2xT_k-T_{k-1}
 *     with basis size 8 (Sec. 5.2 "SVE2 predicated vectorization" and "SME
 *     three-stage pipeline");
 *   - forces -dE/dr and effective fields -dE/ds ("both lattice and spin
 *     driving terms", Sec. 5.2);
 *   - the symplectic spin-lattice step with a predictor-corrector spin update
 *     scheduled last (Sec. 3 and Sec. 5.1 "Self-consistent midpoint spin
 *     update"), with finite-temperature baths on lattice and spins (Sec. 8).
 * The paper names these parts without formulas; the exact forms used here are
 * readings of those names, each stated with the function that takes it
 * (descriptor definitions, B A O S A B splitting, implicit-midpoint Rodrigues
 * spin rotation, Philox4x32-10 normals).
 *
 * Everything is the plain definition: the angular channels are the Legendre
 * double sums over neighbour pairs, derivatives are written out by calculus,
 * neighbour sets are recomputed at every evaluation, sums run in atom order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NR 9      /* radial-set functions n = 0..8            */
#define NA 7      /* angular-set functions n = 0..6           */
#define LMAX 4    /* Legendre orders l = 1..4                 */
#define NB 9      /* Chebyshev basis functions k = 0..8       */
#define NH 64     /* hidden tanh units per species            */
#define ND 102    /* descriptor length                        */

/* descriptor layout */
#define D_R 0
#define D_A 9
#define D_OS 37
#define D_EX 38
#define D_DM 47
#define D_AN 56
#define D_SI 65
#define D_SA 74

/* parameter layout (15,438 doubles) */
#define P_CR 0
#define P_CA 324
#define P_CEX 576
#define P_CDM 900
#define P_CAN 1224
#define P_CSI 1548
#define P_CSA 1872
#define P_MLP 2124
#define P_MLP_STRIDE 6657
#define N_PARAMS 15438

/* physical constants (metal units: A, eV, fs, u, K, T) */
#define KAPPA 9.648533212e-3
#define KB 8.617333262e-5
#define HBAR 0.6582119569
#define MUB 5.7883818060e-5

static const double MASS[2] = {55.845, 72.630};

/* Coulomb constant e^2/(4 pi eps0) in eV A and the Bohr radius in A (CODATA) */
#define KCOUL 14.399645
#define ABOHR 0.529177210903

/* ------------------------------------------------------------------------- */
/* neighbour sets                                                            */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    int *off;      /* [n+1] CSR offsets                   */
    int *j;        /* neighbour index, ascending per atom */
    double *d;     /* [.][3] d_ij = r_j - r_i (min image) */
    double *r;     /* |d_ij|                              */
} nlist_t;

static void nl_free(nlist_t *nl) {
    free(nl->off); free(nl->j); free(nl->d); free(nl->r);
    memset(nl, 0, sizeof(*nl));
}

static void min_image(const double *pi, const double *pj, const double *box,
                      const int *pbc, double d[3]) {
    for (int a = 0; a < 3; a++) {
        double x = pj[a] - pi[a];
        if (pbc[a]) x -= box[a] * nearbyint(x / box[a]);
        d[a] = x;
    }
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Candidate sets per atom: all atoms (brute force) or the 27 cells around the
 * atom's cell (cells at least rc wide). Either way each candidate is then
 * tested by the same minimum-image distance, so both give the same set. */
static int build_nl(int n, const double *pos, const double *box, const int *pbc,
                    double rc, int use_cells, nlist_t *nl) {
    int nc[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, ext[3];
    for (int a = 0; a < 3; a++) {
        if (pbc[a]) {
            ext[a] = box[a];
            nc[a] = (int)floor(box[a] / rc);
        } else {
            double mn = pos[a], mx = pos[a];
            for (int i = 1; i < n; i++) {
                if (pos[3 * i + a] < mn) mn = pos[3 * i + a];
                if (pos[3 * i + a] > mx) mx = pos[3 * i + a];
            }
            lo[a] = mn;
            ext[a] = (mx - mn) * (1 + 1e-12) + 1e-9;
            nc[a] = (int)floor(ext[a] / rc);
        }
        if (nc[a] < 1) nc[a] = 1;
        if (pbc[a] && nc[a] < 3) use_cells = 0;
    }
    int ncell = nc[0] * nc[1] * nc[2];
    int *cell_of = NULL, *cstart = NULL, *cidx = NULL;
    if (use_cells) {
        cell_of = malloc(sizeof(int) * n);
        cstart = calloc(ncell + 1, sizeof(int));
        cidx = malloc(sizeof(int) * n);
        for (int i = 0; i < n; i++) {
            int c[3];
            for (int a = 0; a < 3; a++) {
                double x = pos[3 * i + a] - lo[a];
                if (pbc[a]) x -= box[a] * floor(x / box[a]);
                int k = (int)floor(x / ext[a] * nc[a]);
                if (k < 0) k = 0;
                if (k >= nc[a]) k = nc[a] - 1;
                c[a] = k;
            }
            cell_of[i] = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
            cstart[cell_of[i] + 1]++;
        }
        for (int c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
        int *fill = malloc(sizeof(int) * ncell);
        memcpy(fill, cstart, sizeof(int) * ncell);
        for (int i = 0; i < n; i++) cidx[fill[cell_of[i]]++] = i;
        free(fill);
    }

    int *cnt = calloc(n, sizeof(int));
    int **lists = malloc(sizeof(int *) * n);
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        int cap = 256, m = 0;
        int *cand = malloc(sizeof(int) * cap);
        if (!use_cells) {
            for (int j = 0; j < n; j++) {
                if (m == cap) { cap *= 2; cand = realloc(cand, sizeof(int) * cap); }
                cand[m++] = j;
            }
        } else {
            int ci = cell_of[i];
            int c0 = ci / (nc[1] * nc[2]), c1 = (ci / nc[2]) % nc[1], c2 = ci % nc[2];
            for (int dx = -1; dx <= 1; dx++)
            for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
                int cc[3] = {c0 + dx, c1 + dy, c2 + dz}, ok = 1;
                for (int a = 0; a < 3; a++) {
                    if (cc[a] < 0 || cc[a] >= nc[a]) {
                        if (pbc[a]) cc[a] = (cc[a] + nc[a]) % nc[a];
                        else ok = 0;
                    }
                }
                if (!ok) continue;
                int c = (cc[0] * nc[1] + cc[1]) * nc[2] + cc[2];
                for (int q = cstart[c]; q < cstart[c + 1]; q++) {
                    if (m == cap) { cap *= 2; cand = realloc(cand, sizeof(int) * cap); }
                    cand[m++] = cidx[q];
                }
            }
            qsort(cand, m, sizeof(int), cmp_int);
        }
        int k = 0;
        for (int q = 0; q < m; q++) {
            int j = cand[q];
            if (j == i) continue;
            double d[3];
            min_image(pos + 3 * i, pos + 3 * j, box, pbc, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc * rc) cand[k++] = j;
        }
        lists[i] = cand;
        cnt[i] = k;
    }
    nl->n = n;
    nl->off = malloc(sizeof(int) * (n + 1));
    nl->off[0] = 0;
    for (int i = 0; i < n; i++) nl->off[i + 1] = nl->off[i] + cnt[i];
    int tot = nl->off[n];
    nl->j = malloc(sizeof(int) * (tot + 1));
    nl->d = malloc(sizeof(double) * 3 * (tot + 1));
    nl->r = malloc(sizeof(double) * (tot + 1));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        for (int q = 0; q < cnt[i]; q++) {
            int s = nl->off[i] + q, j = lists[i][q];
            nl->j[s] = j;
            min_image(pos + 3 * i, pos + 3 * j, box, pbc, nl->d + 3 * s);
            double *d = nl->d + 3 * s;
            nl->r[s] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
        free(lists[i]);
    }
    free(lists); free(cnt); free(cell_of); free(cstart); free(cidx);
    return fail;
}

/* ------------------------------------------------------------------------- */
/* radial functions and Legendre polynomials                                 */
/* ------------------------------------------------------------------------- */

/* f_k(r) = (T_k(x)+1)/2 * f_c(r), x = 2(r/rc-1)^2-1, f_c = (1+cos(pi r/rc))/2;
 * zero at and beyond rc. Derivatives by the chain rule, with
 * T'_{k+1} = 2 T_k + 2x T'_k - T'_{k-1} from differentiating the recurrence. */
static void basis(double r, double rc, double f[NB], double df[NB]) {
    if (r >= rc) {
        for (int k = 0; k < NB; k++) { f[k] = 0; df[k] = 0; }
        return;
    }
    double fc = 0.5 * (1.0 + cos(M_PI * r / rc));
    double dfc = -0.5 * M_PI / rc * sin(M_PI * r / rc);
    double u = r / rc - 1.0;
    double x = 2.0 * u * u - 1.0;
    double dxdr = 4.0 * u / rc;
    double T[NB], dT[NB];
    T[0] = 1.0; T[1] = x;
    dT[0] = 0.0; dT[1] = 1.0;
    for (int k = 1; k + 1 < NB; k++) {
        T[k + 1] = 2.0 * x * T[k] - T[k - 1];
        dT[k + 1] = 2.0 * T[k] + 2.0 * x * dT[k] - dT[k - 1];
    }
    for (int k = 0; k < NB; k++) {
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        df[k] = 0.5 * dT[k] * dxdr * fc + 0.5 * (T[k] + 1.0) * dfc;
    }
}

/* g_n(r) = sum_k c[tau][n][k] f_k(r) for nn functions */
static void channel(const double *c, int tau, int nn, const double f[NB],
                    const double df[NB], double *g, double *dg) {
    for (int n = 0; n < nn; n++) {
        const double *cc = c + (tau * nn + n) * NB;
        double a = 0, b = 0;
        for (int k = 0; k < NB; k++) { a += cc[k] * f[k]; b += cc[k] * df[k]; }
        g[n] = a; dg[n] = b;
    }
}

static void legendre(double x, double P[LMAX + 1], double dP[LMAX + 1]) {
    P[0] = 1; dP[0] = 0;
    P[1] = x; dP[1] = 1;
    P[2] = (3 * x * x - 1) / 2; dP[2] = 3 * x;
    P[3] = (5 * x * x * x - 3 * x) / 2; dP[3] = (15 * x * x - 3) / 2;
    P[4] = (35 * x * x * x * x - 30 * x * x + 3) / 8; dP[4] = (140 * x * x * x - 60 * x) / 8;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}


/* ------------------------------------------------------------------------- */
/* optional short-range repulsion                                            */
/* ------------------------------------------------------------------------- */

/* The universal screened-Coulomb (ZBL) repulsion of Ziegler, Biersack and
 * Littmark (The Stopping and Range of Ions in Solids, 1985):
 *   V(r) = KCOUL Z_i Z_j / r * phi(r/a),  a = 0.8854 a_Bohr / (Z_i^0.23 + Z_j^0.23),
 *   phi(x) = 0.18175 e^{-3.19980x} + 0.50986 e^{-0.94229x}
 *          + 0.28022 e^{-0.40290x} + 0.02817 e^{-0.20162x},
 * switched off between r_inner and r_outer by
 *   S(r) = 1 (r <= r_inner), (1 + cos(pi (r - r_inner)/(r_outer - r_inner)))/2, 0 (r >= r_outer).
 * Returns V S and its derivative in r. Sec. 6 includes an optional
 * short-range pair term in the modeled work of a step without giving its
 * form; this is the one NEP models add for close approach. */
static void zbl_pair(double r, double zi, double zj, double r1, double r2, double *V, double *dV) {
    static const double c[4] = {0.18175, 0.50986, 0.28022, 0.02817};
    static const double e[4] = {3.19980, 0.94229, 0.40290, 0.20162};
    if (r >= r2) { *V = 0.0; *dV = 0.0; return; }
    double a = 0.8854 * ABOHR / (pow(zi, 0.23) + pow(zj, 0.23));
    double phi = 0.0, dphi = 0.0;
    for (int k = 0; k < 4; k++) {
        double t = c[k] * exp(-e[k] * r / a);
        phi += t;
        dphi -= e[k] / a * t;
    }
    double pre = KCOUL * zi * zj;
    double v = pre * phi / r;
    double dv = pre * (dphi / r - phi / (r * r));
    double s = 1.0, ds = 0.0;
    if (r > r1) {
        double w = M_PI / (r2 - r1);
        s = 0.5 * (1.0 + cos(w * (r - r1)));
        ds = -0.5 * w * sin(w * (r - r1));
    }
    *V = v * s;
    *dV = dv * s + v * ds;
}

/* ------------------------------------------------------------------------- */
/* model context                                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    const int *type;
    const double *pos;
    double *spin;          /* copy, zero rows on non-magnetic atoms */
    const double *box;
    const int *pbc;
    const double *p;       /* parameters */
    double rcR, rcA;
    int act;               /* 0 tanh, 1 identity (linear read-out, tests only) */
    const double *zbl;     /* short-range term {Z_0, Z_1, r_inner, r_outer}, or NULL */
    const double *landau;  /* onsite moment-length term {a, b} of spin carriers, or NULL */
    nlist_t nl;            /* neighbours within rcR */
    struct nb_s **env;     /* optional per-atom environments (spin step only) */
    int *env_m;
} ctx_t;


/* ------------------------------------------------------------------------- */
/* per-atom neighbour environment                                            */
/* ------------------------------------------------------------------------- */

/* Values of one neighbour j of atom i that the sums below reuse: direction,
 * distance, spin products and the channel functions at r_ij. Computing them
 * once per (i, j) instead of inside every double-sum iteration changes no
 * arithmetic. */
typedef struct nb_s {
    int j, slot, ang;                 /* ang: r_ij < rcA                      */
    double r, rh[3], sig;             /* sig = s_i.s_j                        */
    double gR[NR], dgR[NR], gEX[NR], dgEX[NR], gDM[NR], dgDM[NR];
    double gAN[NR], dgAN[NR], gSI[NR], dgSI[NR];
    double gA[NA], dgA[NA], gS[NA], dgS[NA];
} nb_t;

static int tau_of(const ctx_t *C, int i, int j) { return 2 * C->type[i] + C->type[j]; }

/* environment of atom i: neighbours with r_ij < rcR, in list order */
static int environment(const ctx_t *C, int i, nb_t **out) {
    const nlist_t *nl = &C->nl;
    const double *p = C->p;
    int o = nl->off[i], m = nl->off[i + 1] - o, k = 0;
    nb_t *e = malloc(sizeof(nb_t) * (m + 1));
    double f[NB], df[NB];
    for (int q = 0; q < m; q++) {
        int s = o + q;
        double r = nl->r[s];
        if (r >= C->rcR) continue;
        nb_t *b = e + k++;
        b->j = nl->j[s];
        b->slot = q;
        b->r = r;
        for (int a = 0; a < 3; a++) b->rh[a] = nl->d[3 * s + a] / r;
        b->sig = dot3(C->spin + 3 * i, C->spin + 3 * b->j);
        int tau = tau_of(C, i, b->j);
        basis(r, C->rcR, f, df);
        channel(p + P_CR, tau, NR, f, df, b->gR, b->dgR);
        channel(p + P_CEX, tau, NR, f, df, b->gEX, b->dgEX);
        channel(p + P_CDM, tau, NR, f, df, b->gDM, b->dgDM);
        channel(p + P_CAN, tau, NR, f, df, b->gAN, b->dgAN);
        channel(p + P_CSI, tau, NR, f, df, b->gSI, b->dgSI);
        b->ang = r < C->rcA;
        basis(r, C->rcA, f, df);    /* zero beyond rcA */
        channel(p + P_CA, tau, NA, f, df, b->gA, b->dgA);
        channel(p + P_CSA, tau, NA, f, df, b->gS, b->dgS);
    }
    *out = e;
    return k;
}

/* Environments are cached only while positions stay fixed (the spin step);
 * the cached spin products are not used there. */
static int env_get(const ctx_t *C, int i, nb_t **e) {
    if (C->env && C->env[i]) { *e = C->env[i]; return C->env_m[i]; }
    return environment(C, i, e);
}
static void env_put(const ctx_t *C, int i, nb_t *e) {
    if (!(C->env && C->env[i])) free(e);
}
static void env_cache(ctx_t *C) {
    C->env = calloc(C->n, sizeof(nb_t *));
    C->env_m = calloc(C->n, sizeof(int));
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < C->n; i++)
        if (C->type[i] == 0) C->env_m[i] = environment(C, i, &C->env[i]);
}

/* ------------------------------------------------------------------------- */
/* descriptor of one atom (plain definitions)                                */
/* ------------------------------------------------------------------------- */

static void descriptor_atom(const ctx_t *C, int i, double *q) {
    const double *si = C->spin + 3 * i;
    memset(q, 0, sizeof(double) * ND);
    q[D_OS] = dot3(si, si);
    nb_t *e;
    int m = environment(C, i, &e);
    for (int t = 0; t < m; t++) {
        const nb_t *b = e + t;
        const double *sj = C->spin + 3 * b->j;
        double c[3];
        cross3(si, sj, c);
        double dm = dot3(b->rh, c), a = dot3(si, b->rh), bb = dot3(sj, b->rh);
        for (int n = 0; n < NR; n++) {
            q[D_R + n] += b->gR[n];
            q[D_EX + n] += b->gEX[n] * b->sig;
            q[D_DM + n] += b->gDM[n] * dm;
            q[D_AN + n] += b->gAN[n] * a * bb;
            q[D_SI + n] += b->gSI[n] * a * a;
        }
    }
    /* angular and spin-angular: Legendre double sums over neighbour pairs
     * (j,k) inside rcA, j and k independent, j == k included */
    double P[LMAX + 1], dP[LMAX + 1];
    for (int t = 0; t < m; t++) {
        const nb_t *bj = e + t;
        if (!bj->ang) continue;
        for (int u = 0; u < m; u++) {
            const nb_t *bk = e + u;
            if (!bk->ang) continue;
            legendre(dot3(bj->rh, bk->rh), P, dP);
            for (int n = 0; n < NA; n++)
                for (int l = 1; l <= LMAX; l++) {
                    q[D_A + 4 * n + l - 1] += bj->gA[n] * bk->gA[n] * P[l];
                    q[D_SA + 4 * n + l - 1] += bj->gA[n] * bk->gS[n] * bk->sig * P[l];
                }
        }
    }
    free(e);
}

/* per-species read-out E_i = b1 + sum_h w1_h act(b0_h + sum_d W0_hd q_d) and
 * its gradient Fp_d = dE_i/dq_d */
static double mlp_atom(const ctx_t *C, int t, const double *q, double *Fp) {
    const double *W0 = C->p + P_MLP + t * P_MLP_STRIDE;
    const double *b0 = W0 + NH * ND;
    const double *w1 = b0 + NH;
    const double *b1 = w1 + NH;
    double E = b1[0];
    double gz[NH];
    for (int h = 0; h < NH; h++) {
        double z = b0[h];
        for (int d = 0; d < ND; d++) z += W0[h * ND + d] * q[d];
        double a = C->act ? z : tanh(z);
        E += w1[h] * a;
        gz[h] = w1[h] * (C->act ? 1.0 : (1.0 - a * a));
    }
    if (Fp) {
        for (int d = 0; d < ND; d++) {
            double s = 0;
            for (int h = 0; h < NH; h++) s += W0[h * ND + d] * gz[h];
            Fp[d] = s;
        }
    }
    return E;
}

/* ------------------------------------------------------------------------- */
/* derivatives of one atom's energy                                           */
/*   G[slot]   = dE_i/dd_ij  (d_ij = r_j - r_i), all listed slots            */
/*   hnb[slot] = dE_i/ds_j                                                    */
/*   hown      = dE_i/ds_i                                                    */
/* ------------------------------------------------------------------------- */

static void backward_atom(const ctx_t *C, int i, const double *Fp, double *G,
                          double *hnb, double *hown) {
    const nlist_t *nl = &C->nl;
    const double *si = C->spin + 3 * i;
    int nslot = nl->off[i + 1] - nl->off[i];
    memset(G, 0, sizeof(double) * 3 * nslot);
    memset(hnb, 0, sizeof(double) * 3 * nslot);
    for (int a = 0; a < 3; a++) hown[a] = 2.0 * Fp[D_OS] * si[a];
    if (C->landau && C->type[i] == 0) {
        double r2 = dot3(si, si), k = 2.0 * C->landau[0] + 4.0 * C->landau[1] * r2;
        for (int a = 0; a < 3; a++) hown[a] += k * si[a];
    }
    /* short-range repulsion: E_i holds V(r_ij)/2, dr_ij/dd_ij = rhat_ij */
    if (C->zbl) {
        for (int q = 0; q < nslot; q++) {
            int s = nl->off[i] + q, j = nl->j[s];
            double V, dV, r = nl->r[s];
            zbl_pair(r, C->zbl[C->type[i]], C->zbl[C->type[j]], C->zbl[2], C->zbl[3], &V, &dV);
            for (int a = 0; a < 3; a++) G[3 * q + a] += 0.5 * dV * nl->d[3 * s + a] / r;
        }
    }
    nb_t *e;
    int m = environment(C, i, &e);
    for (int t = 0; t < m; t++) {
        const nb_t *b = e + t;
        const double *sj = C->spin + 3 * b->j;
        const double *rh = b->rh;
        double r = b->r, ss = b->sig;
        double *Gq = G + 3 * b->slot, *hq = hnb + 3 * b->slot;
        double c[3], sjxr[3], rxsi[3];
        cross3(si, sj, c);
        cross3(sj, rh, sjxr);
        cross3(rh, si, rxsi);
        double w = dot3(rh, c), a = dot3(si, rh), bb = dot3(sj, rh);
        for (int n = 0; n < NR; n++) {
            double FR = Fp[D_R + n], FE = Fp[D_EX + n], FD = Fp[D_DM + n];
            double FA = Fp[D_AN + n], FS = Fp[D_SI + n];
            for (int x = 0; x < 3; x++) {
                /* radial: g */
                Gq[x] += FR * b->dgR[n] * rh[x];
                /* exchange: g (s_i.s_j) */
                Gq[x] += FE * b->dgEX[n] * ss * rh[x];
                hown[x] += FE * b->gEX[n] * sj[x];
                hq[x] += FE * b->gEX[n] * si[x];
                /* DMI: g rhat.(s_i x s_j) */
                Gq[x] += FD * (b->dgDM[n] * w * rh[x] + b->gDM[n] * (c[x] - w * rh[x]) / r);
                hown[x] += FD * b->gDM[n] * sjxr[x];
                hq[x] += FD * b->gDM[n] * rxsi[x];
                /* anisotropic exchange: g (s_i.rhat)(s_j.rhat) */
                Gq[x] += FA * (b->dgAN[n] * a * bb * rh[x]
                               + b->gAN[n] * (bb * (si[x] - a * rh[x]) + a * (sj[x] - bb * rh[x])) / r);
                hown[x] += FA * b->gAN[n] * bb * rh[x];
                hq[x] += FA * b->gAN[n] * a * rh[x];
                /* single-ion type: g (s_i.rhat)^2 */
                Gq[x] += FS * (b->dgSI[n] * a * a * rh[x] + 2.0 * b->gSI[n] * a * (si[x] - a * rh[x]) / r);
                hown[x] += FS * 2.0 * b->gSI[n] * a * rh[x];
            }
        }
    }
    /* angular and spin-angular double sums, differentiated in d_ij (j the
     * outer index) through both positions j takes in the pair sum */
    double P[LMAX + 1], dP[LMAX + 1];
    for (int t = 0; t < m; t++) {
        const nb_t *bj = e + t;
        if (!bj->ang) continue;
        const double *sj = C->spin + 3 * bj->j;
        double *Gq = G + 3 * bj->slot, *hq = hnb + 3 * bj->slot;
        for (int u = 0; u < m; u++) {
            const nb_t *bb = e + u;
            if (!bb->ang) continue;
            double cth = dot3(bj->rh, bb->rh);
            legendre(cth, P, dP);
            double perp[3];   /* d(rhat_j . rhat_b)/d d_ij */
            for (int x = 0; x < 3; x++) perp[x] = (bb->rh[x] - cth * bj->rh[x]) / bj->r;
            for (int n = 0; n < NA; n++)
                for (int l = 1; l <= LMAX; l++) {
                    double FA = Fp[D_A + 4 * n + l - 1], FS = Fp[D_SA + 4 * n + l - 1];
                    /* q^A = sum_j sum_b gA_j gA_b P(c_jb): symmetric, factor 2 */
                    double tA = 2.0 * FA * bj->dgA[n] * bb->gA[n] * P[l];
                    double uA = 2.0 * FA * bj->gA[n] * bb->gA[n] * dP[l];
                    /* q^sa = sum_a sum_b gA_a gS_b sig_b P(c_ab): j as a, then j as b */
                    double tS = FS * (bj->dgA[n] * bb->gS[n] * bb->sig + bb->gA[n] * bj->dgS[n] * bj->sig) * P[l];
                    double uS = FS * (bj->gA[n] * bb->gS[n] * bb->sig + bb->gA[n] * bj->gS[n] * bj->sig) * dP[l];
                    double h = FS * bb->gA[n] * bj->gS[n] * P[l];
                    for (int x = 0; x < 3; x++) {
                        Gq[x] += (tA + tS) * bj->rh[x] + (uA + uS) * perp[x];
                        /* dq^sa/ds_j = sum_a gA_a gS_j P(c_aj) s_i, and the
                         * same terms times s_j sum to dq^sa/ds_i */
                        hq[x] += h * si[x];
                        hown[x] += h * sj[x];
                    }
                }
        }
    }
    free(e);
}

/* dE_i/ds_i without the onsite and single-ion channels (the only ones in
 * which s_i appears together with itself) */
static void spin_grad_own_fixed(const ctx_t *C, int i, const double *Fp, double h[3]) {
    h[0] = h[1] = h[2] = 0.0;
    nb_t *e;
    int m = env_get(C, i, &e);
    for (int t = 0; t < m; t++) {
        const nb_t *b = e + t;
        const double *sj = C->spin + 3 * b->j;
        double sjxr[3];
        cross3(sj, b->rh, sjxr);
        double bb = dot3(sj, b->rh);
        for (int n = 0; n < NR; n++)
            for (int x = 0; x < 3; x++)
                h[x] += Fp[D_EX + n] * b->gEX[n] * sj[x] + Fp[D_DM + n] * b->gDM[n] * sjxr[x]
                        + Fp[D_AN + n] * b->gAN[n] * bb * b->rh[x];
    }
    double P[LMAX + 1], dP[LMAX + 1];
    for (int t = 0; t < m; t++) {
        const nb_t *ba = e + t;
        if (!ba->ang) continue;
        for (int u = 0; u < m; u++) {
            const nb_t *bb = e + u;
            if (!bb->ang) continue;
            legendre(dot3(ba->rh, bb->rh), P, dP);
            const double *sb = C->spin + 3 * bb->j;
            for (int n = 0; n < NA; n++)
                for (int l = 1; l <= LMAX; l++) {
                    double v = Fp[D_SA + 4 * n + l - 1] * ba->gA[n] * bb->gS[n] * P[l];
                    for (int x = 0; x < 3; x++) h[x] += v * sb[x];
                }
        }
    }
    env_put(C, i, e);
}

/* dE_k/ds_i for a neighbour k of i */
static void spin_grad_onto(const ctx_t *C, int k, int i, const double *Fp, double h[3]) {
    h[0] = h[1] = h[2] = 0.0;
    nb_t *e;
    int m = env_get(C, k, &e);
    const double *sk = C->spin + 3 * k;
    int ti = -1;
    for (int t = 0; t < m; t++)
        if (e[t].j == i) ti = t;
    if (ti < 0) { env_put(C, k, e); return; }
    const nb_t *bi = e + ti;
    double rxsk[3];
    cross3(bi->rh, sk, rxsk);
    double a = dot3(sk, bi->rh);
    for (int n = 0; n < NR; n++)
        for (int x = 0; x < 3; x++)
            h[x] += Fp[D_EX + n] * bi->gEX[n] * sk[x] + Fp[D_DM + n] * bi->gDM[n] * rxsk[x]
                    + Fp[D_AN + n] * bi->gAN[n] * a * bi->rh[x];
    if (bi->ang) {
        double P[LMAX + 1], dP[LMAX + 1];
        for (int t = 0; t < m; t++) {
            const nb_t *ba = e + t;
            if (!ba->ang) continue;
            legendre(dot3(ba->rh, bi->rh), P, dP);
            for (int n = 0; n < NA; n++)
                for (int l = 1; l <= LMAX; l++) {
                    double v = Fp[D_SA + 4 * n + l - 1] * ba->gA[n] * bi->gS[n] * P[l];
                    for (int x = 0; x < 3; x++) h[x] += v * sk[x];
                }
        }
    }
    env_put(C, k, e);
}

/* ------------------------------------------------------------------------- */
/* full evaluation                                                           */
/* ------------------------------------------------------------------------- */

typedef struct {
    double E_nep, E_z;
    double *Ei, *F, *H, *q, *Fp;    /* optional outputs ([n], [n][3], [n][3], [n][ND], [n][ND]) */
} evalout_t;

static void ctx_init(ctx_t *C, int n, const int *type, const double *pos, const double *spin,
                     const double *box, const int *pbc, const double *p, double rcR, double rcA,
                     int act, int use_cells) {
    C->n = n; C->type = type; C->pos = pos; C->box = box; C->pbc = pbc; C->p = p;
    C->rcR = rcR; C->rcA = rcA; C->act = act;
    C->zbl = NULL;
    C->landau = NULL;
    C->spin = malloc(sizeof(double) * 3 * (n + 1));
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) C->spin[3 * i + a] = type[i] == 0 ? spin[3 * i + a] : 0.0;
    memset(&C->nl, 0, sizeof(C->nl));
    C->env = NULL;
    C->env_m = NULL;
    build_nl(n, pos, box, pbc, rcR, use_cells, &C->nl);
}

static void ctx_free(ctx_t *C) {
    if (C->env) {
        for (int i = 0; i < C->n; i++) free(C->env[i]);
        free(C->env);
        free(C->env_m);
    }
    free(C->spin);
    nl_free(&C->nl);
}

/* descriptors and read-out for all atoms: q, Fp, E_i */
static double forward_all(const ctx_t *C, double *q, double *Fp, double *Ei) {
    int n = C->n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; i++) {
        descriptor_atom(C, i, q + (size_t)ND * i);
        Ei[i] = mlp_atom(C, C->type[i], q + (size_t)ND * i, Fp + (size_t)ND * i);
        /* onsite moment-length term a |s|^2 + b |s|^4 of a spin carrier */
        if (C->landau && C->type[i] == 0) {
            double r2 = dot3(C->spin + 3 * i, C->spin + 3 * i);
            Ei[i] += C->landau[0] * r2 + C->landau[1] * r2 * r2;
        }
        /* short-range repulsion: half of each pair's energy to each atom */
        if (C->zbl) {
            const nlist_t *nl = &C->nl;
            for (int s = nl->off[i]; s < nl->off[i + 1]; s++) {
                int j = nl->j[s];
                double V, dV;
                zbl_pair(nl->r[s], C->zbl[C->type[i]], C->zbl[C->type[j]], C->zbl[2], C->zbl[3], &V, &dV);
                Ei[i] += 0.5 * V;
            }
        }
    }
    double E = 0;
    for (int i = 0; i < n; i++) E += Ei[i];
    return E;
}

static double zeeman(const ctx_t *C, double mu_s, const double *B) {
    double E = 0;
    for (int i = 0; i < C->n; i++)
        if (C->type[i] == 0) E -= mu_s * MUB * dot3(B, C->spin + 3 * i);
    return E;
}

/* forces and fields from Fp (scatter in atom order) */
static void forces_fields(const ctx_t *C, const double *Fp, double mu_s, const double *B,
                          double *F, double *H) {
    int n = C->n, tot = C->nl.off[n];
    double *G = malloc(sizeof(double) * 3 * (tot + 1));
    double *hn = malloc(sizeof(double) * 3 * (tot + 1));
    double *ho = malloc(sizeof(double) * 3 * (n + 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; i++) {
        int o = C->nl.off[i];
        backward_atom(C, i, Fp + (size_t)ND * i, G + 3 * o, hn + 3 * o, ho + 3 * i);
    }
    double *dEds = calloc(3 * (size_t)n, sizeof(double));
    memset(F, 0, sizeof(double) * 3 * n);
    for (int i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++) dEds[3 * i + a] += ho[3 * i + a];
        for (int s = C->nl.off[i]; s < C->nl.off[i + 1]; s++) {
            int j = C->nl.j[s];
            for (int a = 0; a < 3; a++) {
                /* E_i depends on d_ij = r_j - r_i */
                F[3 * i + a] += G[3 * s + a];
                F[3 * j + a] -= G[3 * s + a];
                dEds[3 * j + a] += hn[3 * s + a];
            }
        }
    }
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++)
            H[3 * i + a] = C->type[i] == 0 ? -dEds[3 * i + a] + mu_s * MUB * B[a] : 0.0;
    free(G); free(hn); free(ho); free(dEds);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals  */
/* ------------------------------------------------------------------------- */

static void philox(const uint32_t cin[4], const uint32_t kin[2], uint32_t out[4]) {
    uint32_t c0 = cin[0], c1 = cin[1], c2 = cin[2], c3 = cin[3], k0 = kin[0], k1 = kin[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* three standard normals for (seed, atom, step, stream): counter =
 * (atom, step lo, step hi, stream*256 + draw), key = (seed lo, seed hi);
 * u1 = 1 - (53-bit word)*2^-53 in (0,1], u2 = (53-bit word)*2^-53 */
static void normals3(uint64_t seed, uint32_t atom, uint64_t step, uint32_t stream, double xi[3]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double z[4];
    for (uint32_t draw = 0; draw < 2; draw++) {
        uint32_t ctr[4] = {atom, (uint32_t)step, (uint32_t)(step >> 32), stream * 256u + draw};
        uint32_t x[4];
        philox(ctr, key, x);
        uint64_t a = (((uint64_t)x[0] << 32) | x[1]) >> 11;
        uint64_t b = (((uint64_t)x[2] << 32) | x[3]) >> 11;
        double u1 = 1.0 - (double)a * 0x1.0p-53;
        double u2 = (double)b * 0x1.0p-53;
        double rad = sqrt(-2.0 * log(u1));
        z[2 * draw] = rad * cos(2.0 * M_PI * u2);
        z[2 * draw + 1] = rad * sin(2.0 * M_PI * u2);
    }
    xi[0] = z[0]; xi[1] = z[1]; xi[2] = z[2];
}

/* ------------------------------------------------------------------------- */
/* exported evaluation API                                                   */
/* ------------------------------------------------------------------------- */

int or_n_params(void) { return N_PARAMS; }
int or_n_desc(void) { return ND; }

int or_neighbors(int n, const double *pos, const double *box, const int *pbc, double rc,
                 int use_cells, int maxnb, int *cnt, int *nbr) {
    nlist_t nl;
    memset(&nl, 0, sizeof(nl));
    build_nl(n, pos, box, pbc, rc, use_cells, &nl);
    int over = 0;
    for (int i = 0; i < n; i++) {
        int m = nl.off[i + 1] - nl.off[i];
        cnt[i] = m;
        if (m > maxnb) { over = 1; m = maxnb; }
        for (int q = 0; q < m; q++) nbr[(size_t)i * maxnb + q] = nl.j[nl.off[i] + q];
    }
    nl_free(&nl);
    return over ? -1 : 0;
}

/* E = E_NEP (+ E_Zeeman reported separately); all outputs optional. zbl:
 * {Z_0, Z_1, r_inner, r_outer} of the short-range term, or NULL (off, also
 * when r_outer <= 0); landau: {a, b} of the onsite moment-length term, or
 * NULL. E_NEP and E_i include both; H includes the latter. */
int or_eval(int n, const int *type, const double *pos, const double *spin, const double *box,
            const int *pbc, const double *params, double rcR, double rcA, int act,
            double mu_s, const double *B, double *E_nep, double *E_z, double *Ei, double *F,
            double *H, double *q_out, double *Fp_out, const double *zbl, const double *landau) {
    ctx_t C;
    ctx_init(&C, n, type, pos, spin, box, pbc, params, rcR, rcA, act, n > 4096);
    if (zbl && zbl[3] > 0) C.zbl = zbl;
    if (landau && (landau[0] != 0 || landau[1] != 0)) C.landau = landau;
    double *q = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Fp = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Ea = malloc(sizeof(double) * (n + 1));
    double E = forward_all(&C, q, Fp, Ea);
    if (E_nep) *E_nep = E;
    if (E_z) *E_z = zeeman(&C, mu_s, B);
    if (Ei) memcpy(Ei, Ea, sizeof(double) * n);
    if (q_out) memcpy(q_out, q, sizeof(double) * ND * (size_t)n);
    if (Fp_out) memcpy(Fp_out, Fp, sizeof(double) * ND * (size_t)n);
    if (F || H) {
        double *Fx = F ? F : malloc(sizeof(double) * 3 * (size_t)n);
        double *Hx = H ? H : malloc(sizeof(double) * 3 * (size_t)n);
        forces_fields(&C, Fp, mu_s, B, Fx, Hx);
        if (!F) free(Fx);
        if (!H) free(Hx);
    }
    free(q); free(Fp); free(Ea);
    ctx_free(&C);
    return 0;
}

int or_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    philox(ctr, key, out);
    return 0;
}

int or_normals(uint64_t seed, uint32_t atom, uint64_t step, uint32_t stream, double *xi) {
    normals3(seed, atom, step, stream, xi);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* the spin-lattice step                                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    double dt, T0, T1, B0[3], B1[3], alpha, gammaL, mu_s, mid_tol, rcR, rcA;
    int64_t n_ramp;
    uint64_t seed;
    int ensemble, K_corr, mid_cap, act, sequential;
    /* self-consistent midpoint (sc_tol > 0): corrector passes are repeated
     * until max over spins of |S^(p) - S^(p-1)| <= sc_tol, at most sc_max
     * passes after the predictor; K_corr is then not used */
    int sc_max;
    double sc_tol;
    /* accelerated variant (sc_depth > 0): Anderson mixing over the last
     * sc_depth differences of residuals, Tikhonov-regularised by sc_reg times
     * the mean diagonal of their Gram matrix */
    int sc_depth;
    double sc_reg;
    /* structural-only model (the standard NEP without magnetic channels): no
     * spins, the step is B A O A B; masses per species (u), 0 = Fe/Ge */
    int structural;
    double mass[2];
    /* short-range repulsion {Z_0, Z_1, r_inner, r_outer}; off when r_outer <= 0 */
    double zbl[4];
    /* onsite moment-length term a |s|^2 + b |s|^4 on spin carriers (off when
     * both are 0), and the moment-length (longitudinal) fluctuations: lsf = 1
     * replaces the transverse bath (alpha unused) by the Langevin dynamics
     * ds/dt = (h x s)/hbar + (lsf_gamma/hbar) h + noise, whose damping and
     * noise also change |s| */
    double landau[2];
    int lsf;
    double lsf_gamma;
} or_step_params;

typedef struct {
    double step, E_nep, E_kin, E_z, T_lat, T_spin, M[3];
    double passes;   /* sweeps of the spin step (predictor + correctors)      */
    double change;   /* max |g - x| of its last pass                         */
    double capped;   /* spin rotations of the step (all passes) that stopped
                        at mid_cap without meeting mid_tol                   */
    double s_len;    /* mean |s| over the spin carriers                       */
} or_obs;

/* Anderson mixing (type II) for a fixed point x = g(x) of dimension n.
 * Given the current residual f = g(x_k) - x_k and the value g = g(x_k), and
 * m columns of differences dF[a] = f_j - f_{j-1}, dG[a] = g_j - g_{j-1}
 * (column a at dF + a*n), the coefficients minimise
 * |f - sum_a gam_a dF[a]|^2 + lam |gam|^2, lam = reg * trace(dF^T dF) / m,
 * and the next iterate is x_{k+1} = g - sum_a gam_a dG[a]. The normal
 * equations are solved by Cholesky; without a positive definite system (no
 * differences, or a pivot below 1e-13 of its diagonal entry: a column in the
 * span of the others, possible with reg = 0) the step is the plain one,
 * x_{k+1} = g. Returns the number of columns used (0 or m). */
int or_anderson_mix(int n, int m, const double *dF, const double *dG, const double *f, const double *g,
                    double reg, double *x_next, double *gam_out) {
    double G[8][8], r[8], L[8][8], y[8], gam[8];
    int used = 0;
    if (m > 8) m = 8;
    for (int a = 0; a < m; a++) {
        for (int b = 0; b < m; b++) {
            double acc = 0;
            for (int i = 0; i < n; i++) acc += dF[(size_t)a * n + i] * dF[(size_t)b * n + i];
            G[a][b] = acc;
        }
        double acc = 0;
        for (int i = 0; i < n; i++) acc += dF[(size_t)a * n + i] * f[i];
        r[a] = acc;
    }
    double tr = 0;
    for (int a = 0; a < m; a++) tr += G[a][a];
    if (m > 0 && tr > 0) {
        const double lam = reg * tr / m;
        int ok = 1;
        for (int a = 0; a < m && ok; a++) {
            for (int b = 0; b <= a; b++) {
                double v = G[a][b] + (a == b ? lam : 0.0);
                for (int c = 0; c < b; c++) v -= L[a][c] * L[b][c];
                if (a == b) {
                    /* a column (numerically) in the span of the earlier ones */
                    if (!(v > 1e-13 * (G[a][a] + lam))) { ok = 0; break; }
                    L[a][a] = sqrt(v);
                } else {
                    L[a][b] = v / L[b][b];
                }
            }
        }
        if (ok) {
            for (int a = 0; a < m; a++) {
                double v = r[a];
                for (int c = 0; c < a; c++) v -= L[a][c] * y[c];
                y[a] = v / L[a][a];
            }
            for (int a = m - 1; a >= 0; a--) {
                double v = y[a];
                for (int c = a + 1; c < m; c++) v -= L[c][a] * gam[c];
                gam[a] = v / L[a][a];
            }
            used = m;
        }
    }
    for (int a = 0; a < m; a++)
        if (gam_out) gam_out[a] = used ? gam[a] : 0.0;
    for (int i = 0; i < n; i++) {
        double v = g[i];
        for (int a = 0; a < used; a++) v -= gam[a] * dG[(size_t)a * n + i];
        x_next[i] = v;
    }
    return used;
}

/* field of the frozen-Fp magnetic energy on spin i, split into the part that
 * does not involve s_i (bilinear terms with neighbour spins) and the part
 * linear in s_i itself (onsite and single-ion channels), so that the latter
 * can be evaluated at each midpoint iterate */
static void hlin_fixed(const ctx_t *C, const double *Fps, int i, double h[3]) {
    const nlist_t *nl = &C->nl;
    double t[3];
    /* own descriptor, without the onsite and single-ion terms */
    spin_grad_own_fixed(C, i, Fps + (size_t)ND * i, h);
    /* neighbours' descriptors: dE_k/ds_i for every spin-carrying k within rcR */
    for (int s = nl->off[i]; s < nl->off[i + 1]; s++) {
        int k = nl->j[s];
        if (C->type[k] != 0 || nl->r[s] >= C->rcR) continue;
        spin_grad_onto(C, k, i, Fps + (size_t)ND * k, t);
        for (int a = 0; a < 3; a++) h[a] += t[a];
    }
    for (int a = 0; a < 3; a++) h[a] = -h[a];
}

/* -d/ds_i of the terms in s_i alone (onsite and single-ion channels, which
 * the frozen Fp makes quadratic, and the exact onsite moment-length term),
 * evaluated at x */
static void hlin_self(const ctx_t *C, const double *Fps, int i, const double *x, double h[3]) {
    for (int a = 0; a < 3; a++) h[a] = -2.0 * Fps[(size_t)ND * i + D_OS] * x[a];
    if (C->landau) {
        double k = 2.0 * C->landau[0] + 4.0 * C->landau[1] * dot3(x, x);
        for (int a = 0; a < 3; a++) h[a] -= k * x[a];
    }
    nb_t *e;
    int m = env_get(C, i, &e);
    for (int t = 0; t < m; t++) {
        double a_ = dot3(x, e[t].rh);
        for (int n = 0; n < NR; n++)
            for (int y = 0; y < 3; y++) h[y] -= Fps[(size_t)ND * i + D_SI + n] * 2.0 * e[t].gSI[n] * a_ * e[t].rh[y];
    }
    env_put(C, i, e);
}

/* one implicit-midpoint Rodrigues rotation of spin s over time tau: the
 * midpoint equation y = G(y), G(y) the rotation of s about the precession
 * vector taken at the midpoint m of s and y (direction of s + y, length
 * |s|), solved by plain iteration until max|G(y) - y| <= mid_tol or mid_cap
 * evaluations; returns the last G(y) and sets *capped when the tolerance was
 * not met */
static void midpoint_rotation(const ctx_t *C, const double *Fps, int i, const double *s, const double *hfix,
                              double tau, const double *Bext, const double *eta, const or_step_params *sp,
                              double *out, int *capped) {
    double y[3] = {s[0], s[1], s[2]}, yn[3];
    double al = sp->lsf ? 0.0 : sp->alpha;
    double len = sp->lsf ? sqrt(dot3(s, s)) : 1.0;
    int conv = 0;
    for (int it = 0; it < sp->mid_cap; it++) {
        double xb[3] = {s[0] + y[0], s[1] + y[1], s[2] + y[2]};
        double nx = sqrt(dot3(xb, xb));
        for (int a = 0; a < 3; a++) xb[a] /= nx;
        if (sp->lsf)
            for (int a = 0; a < 3; a++) xb[a] *= len;
        double hs[3], h[3], xh[3], w[3];
        hlin_self(C, Fps, i, xb, hs);
        for (int a = 0; a < 3; a++) h[a] = hfix[a] + hs[a] + sp->mu_s * MUB * Bext[a] + eta[a];
        cross3(xb, h, xh);
        for (int a = 0; a < 3; a++) w[a] = (h[a] + al * xh[a]) / (1.0 + al * al);
        double wn = sqrt(dot3(w, w));
        if (wn == 0.0) {
            for (int a = 0; a < 3; a++) yn[a] = s[a];
        } else {
            double th = wn * tau / HBAR, sn, cs, omc;
            if (fabs(th) < 1e-8) {
                sn = th - th * th * th / 6.0;
                cs = 1.0 - th * th / 2.0;
                omc = th * th / 2.0;
            } else {
                sn = sin(th);
                cs = cos(th);
                omc = 1.0 - cs;
            }
            double wh[3] = {w[0] / wn, w[1] / wn, w[2] / wn}, wxs[3];
            cross3(wh, s, wxs);
            double ws = dot3(wh, s);
            for (int a = 0; a < 3; a++) yn[a] = s[a] * cs + wxs[a] * sn + wh[a] * ws * omc;
        }
        double diff = 0;
        for (int a = 0; a < 3; a++) {
            double dd = fabs(yn[a] - y[a]);
            if (dd > diff) diff = dd;
            y[a] = yn[a];
        }
        if (diff <= sp->mid_tol) { conv = 1; break; }
    }
    for (int a = 0; a < 3; a++) out[a] = y[a];
    if (!conv) *capped += 1;
}

/* Longitudinal half step of the Langevin dynamics with moment-length
 * fluctuations over time t: s += (gamma t / hbar) h(s) + sqrt(2 gamma kB T t / hbar) xi,
 * h the full frozen-Fp field at s (neighbours, own channels, onsite
 * moment-length term, Zeeman), xi three normals (Euler-Maruyama step of
 * ds = (gamma/hbar) h dt + sqrt(2 gamma kB T / hbar) dW) */
static void lsf_half(const ctx_t *C, const double *Fps, int i, double *s, const double *hfix, double t,
                     const double *Bext, double T, const or_step_params *sp, uint64_t step, uint32_t stream) {
    double hs[3], xi[3] = {0, 0, 0};
    hlin_self(C, Fps, i, s, hs);
    if (T > 0) normals3(sp->seed, (uint32_t)i, step, stream, xi);
    double k = sp->lsf_gamma * t / HBAR, sig = sqrt(2.0 * sp->lsf_gamma * KB * T * t / HBAR);
    for (int a = 0; a < 3; a++) s[a] += k * (hfix[a] + hs[a] + sp->mu_s * MUB * Bext[a]) + sig * xi[a];
}

/* The update of spin i for one visit of its colour (time tau): the implicit-
 * midpoint rotation; with moment-length fluctuations, between two
 * longitudinal half steps (noise streams 2 + 2 visit and 3 + 2 visit, visit 0
 * on the ascending and 1 on the descending pass). */
static void rotate_spin(const ctx_t *C, const double *Fps, int i, double tau, const double *Bext,
                        const double *eta, const or_step_params *sp, double T, int visit, uint64_t step,
                        double *snew, int *capped) {
    double s[3] = {C->spin[3 * i], C->spin[3 * i + 1], C->spin[3 * i + 2]};
    double hfix[3];
    hlin_fixed(C, Fps, i, hfix);
    if (sp->lsf && sp->lsf_gamma > 0) {
        lsf_half(C, Fps, i, s, hfix, 0.5 * tau, Bext, T, sp, step, 2u + 2u * (uint32_t)visit);
        midpoint_rotation(C, Fps, i, s, hfix, tau, Bext, eta, sp, snew, capped);
        lsf_half(C, Fps, i, snew, hfix, 0.5 * tau, Bext, T, sp, step, 3u + 2u * (uint32_t)visit);
    } else {
        midpoint_rotation(C, Fps, i, s, hfix, tau, Bext, eta, sp, snew, capped);
    }
}

static void wrap(int n, double *pos, const double *box, const int *pbc) {
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++)
            if (pbc[a]) pos[3 * i + a] -= box[a] * floor(pos[3 * i + a] / box[a]);
}

/* Run n_steps of the B A O S A B step from (pos, vel, spin, *step).
 * colour[i] >= 0 on Fe (classes 0..ncol-1), -1 on Ge. */
int or_run(int n, const int *type, double *pos, double *vel, double *spin, const double *box,
           const int *pbc, const double *params, const int *colour, int ncol,
           const or_step_params *sp, int64_t *step, int64_t n_steps, or_obs *obs) {
    ctx_t C;
    int use_cells = n > 4096;
    double *q = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Fp = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Ei = malloc(sizeof(double) * (n + 1));
    double *F = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *H = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *Sn = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *Sh = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *eta = calloc(3 * (size_t)(n + 1), sizeof(double));
    double *snew = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    int *cap_of = calloc((size_t)(n + 1), sizeof(int));
    /* self-consistent iteration: the iterate x (end-of-step spins whose
     * midpoint the pass uses) and, for the accelerated variant, the history */
    const int depth = sp->sc_tol > 0 && sp->sc_depth > 0 ? (sp->sc_depth < 8 ? sp->sc_depth : 8) : 0;
    int nfe_all = 0;
    for (int i = 0; i < n; i++) nfe_all += type[i] == 0;
    const size_t nv = 3 * (size_t)nfe_all + 1;
    double *X = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *fk = malloc(sizeof(double) * nv), *gk = malloc(sizeof(double) * nv);
    double *fprev = malloc(sizeof(double) * nv), *gprev = malloc(sizeof(double) * nv);
    double *xnew = malloc(sizeof(double) * nv);
    double *dF = malloc(sizeof(double) * nv * (depth + 1)), *dG = malloc(sizeof(double) * nv * (depth + 1));
    double dt = sp->dt;
    const double mt[2] = {sp->mass[0] > 0 ? sp->mass[0] : MASS[0], sp->mass[1] > 0 ? sp->mass[1] : MASS[1]};
    for (int i = 0; i < n; i++)
        if (sp->structural || type[i] != 0) spin[3 * i] = spin[3 * i + 1] = spin[3 * i + 2] = 0.0;
    double B[3], Bz[3] = {0, 0, 0};
    /* F^0 at the start state */
    {
        double frac = sp->n_ramp > 0 ? (double)(*step < sp->n_ramp ? *step : sp->n_ramp) / sp->n_ramp : 0.0;
        for (int a = 0; a < 3; a++) B[a] = sp->B0[a] + (sp->B1[a] - sp->B0[a]) * frac;
        ctx_init(&C, n, type, pos, spin, box, pbc, params, sp->rcR, sp->rcA, sp->act, use_cells);
        if (sp->zbl[3] > 0) C.zbl = sp->zbl;
        if (sp->landau[0] != 0 || sp->landau[1] != 0) C.landau = sp->landau;
        forward_all(&C, q, Fp, Ei);
        forces_fields(&C, Fp, sp->mu_s, Bz, F, H);
        ctx_free(&C);
    }
    for (int64_t it = 0; it < n_steps; it++) {
        int64_t st = *step;
        double frac = sp->n_ramp > 0 ? (double)(st < sp->n_ramp ? st : sp->n_ramp) / sp->n_ramp : 0.0;
        double T = sp->T0 + (sp->T1 - sp->T0) * frac;
        for (int a = 0; a < 3; a++) B[a] = sp->B0[a] + (sp->B1[a] - sp->B0[a]) * frac;
        /* B: half kick */
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) vel[3 * i + a] += 0.5 * dt * KAPPA * F[3 * i + a] / mt[type[i]];
        /* A: half drift */
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) pos[3 * i + a] += 0.5 * dt * vel[3 * i + a];
        wrap(n, pos, box, pbc);
        /* O: lattice Langevin */
        if (sp->ensemble == 1) {
            double c1 = exp(-sp->gammaL * dt);
            for (int i = 0; i < n; i++) {
                double xi[3];
                normals3(sp->seed, (uint32_t)i, (uint64_t)st, 0, xi);
                double sig = sqrt((1.0 - c1 * c1) * KAPPA * KB * T / mt[type[i]]);
                for (int a = 0; a < 3; a++) vel[3 * i + a] = c1 * vel[3 * i + a] + sig * xi[a];
            }
        }
        int passes = 0, capped = 0;
        double change = 0;
        /* S: spin step at R_mid (none for a structural-only model) */
        if (!sp->structural) {
            double esig = (!sp->lsf && sp->alpha > 0 && T > 0) ? sqrt(2.0 * sp->alpha * KB * T * HBAR / dt) : 0.0;
            for (int i = 0; i < n; i++) {
                double xi[3] = {0, 0, 0};
                if (esig > 0 && type[i] == 0) normals3(sp->seed, (uint32_t)i, (uint64_t)st, 1, xi);
                for (int a = 0; a < 3; a++) eta[3 * i + a] = esig * xi[a];
            }
            memcpy(Sn, spin, sizeof(double) * 3 * n);
            memcpy(Sh, spin, sizeof(double) * 3 * n);
            memcpy(X, spin, sizeof(double) * 3 * n);   /* x^(0) = S^n: the predictor */
            const int self_consistent = sp->sc_tol > 0;
            const int last = self_consistent ? sp->sc_max : sp->K_corr;
            int ncols = 0;
            for (int pc = 0; pc <= last; pc++) {
                /* Fp* at (R_mid, S_hat) */
                ctx_init(&C, n, type, pos, Sh, box, pbc, params, sp->rcR, sp->rcA, sp->act, use_cells);
                if (sp->landau[0] != 0 || sp->landau[1] != 0) C.landau = sp->landau;
                forward_all(&C, q, Fp, Ei);
                /* restart from S^n; C.spin now holds the spins being swept */
                memcpy(C.spin, Sn, sizeof(double) * 3 * n);
                env_cache(&C);
                memset(cap_of, 0, sizeof(int) * (size_t)(n + 1));
                for (int pass = 0; pass < 2; pass++) {
                    for (int cc = 0; cc < ncol; cc++) {
                        int c = pass == 0 ? cc : ncol - 1 - cc;
                        if (sp->sequential) {
                            for (int i = 0; i < n; i++)
                                if (colour[i] == c) {
                                    rotate_spin(&C, Fp, i, 0.5 * dt, B, eta + 3 * i, sp, T, pass, (uint64_t)st,
                                                snew + 3 * i, &capped);
                                    for (int a = 0; a < 3; a++) C.spin[3 * i + a] = snew[3 * i + a];
                                }
                        } else {
    #pragma omp parallel for schedule(dynamic, 8)
                            for (int i = 0; i < n; i++)
                                if (colour[i] == c) rotate_spin(&C, Fp, i, 0.5 * dt, B, eta + 3 * i, sp, T, pass,
                                                                (uint64_t)st, snew + 3 * i, &cap_of[i]);
                            for (int i = 0; i < n; i++)
                                if (colour[i] == c)
                                    for (int a = 0; a < 3; a++) C.spin[3 * i + a] = snew[3 * i + a];
                        }
                    }
                }
                for (int i = 0; i < n; i++) capped += cap_of[i];
                passes = pc + 1;
                /* residual of the pass: g - x, with g the swept spins (for the
                 * plain iteration x is the previous pass's g, S^n for the first) */
                change = 0;
                for (int i = 0; i < n; i++)
                    if (type[i] == 0)
                        for (int a = 0; a < 3; a++) {
                            const double d = fabs(C.spin[3 * i + a] - X[3 * i + a]);
                            if (d > change) change = d;
                        }
                memcpy(spin, C.spin, sizeof(double) * 3 * n);
                ctx_free(&C);
                if (self_consistent && pc >= 1 && change <= sp->sc_tol) break;
                if (pc == last) break;
                /* next iterate: plain, x = g; accelerated, Anderson mixing of the
                 * last depth residual differences */
                if (depth == 0) {
                    memcpy(X, spin, sizeof(double) * 3 * n);
                } else {
                    size_t k = 0;
                    for (int i = 0; i < n; i++)
                        if (type[i] == 0)
                            for (int a = 0; a < 3; a++, k++) {
                                gk[k] = spin[3 * i + a];
                                fk[k] = spin[3 * i + a] - X[3 * i + a];
                            }
                    if (pc >= 1) {
                        /* newest difference in front, the oldest dropped */
                        const int keep = ncols < depth ? ncols : depth - 1;
                        memmove(dF + k, dF, sizeof(double) * k * keep);
                        memmove(dG + k, dG, sizeof(double) * k * keep);
                        for (size_t e = 0; e < k; e++) {
                            dF[e] = fk[e] - fprev[e];
                            dG[e] = gk[e] - gprev[e];
                        }
                        ncols = keep + 1;
                    }
                    memcpy(fprev, fk, sizeof(double) * k);
                    memcpy(gprev, gk, sizeof(double) * k);
                    or_anderson_mix((int)k, ncols, dF, dG, fk, gk, sp->sc_reg, xnew, NULL);
                    k = 0;
                    for (int i = 0; i < n; i++)
                        if (type[i] == 0)
                            for (int a = 0; a < 3; a++, k++) X[3 * i + a] = xnew[k];
                }
                /* S_hat = normalise((S^n + x)/2) on spin-carrying atoms */
                for (int i = 0; i < n; i++) {
                    if (type[i] != 0) continue;
                    double m[3], nn;
                    for (int a = 0; a < 3; a++) m[a] = 0.5 * (Sn[3 * i + a] + X[3 * i + a]);
                    nn = sqrt(dot3(m, m));
                    /* with moment-length fluctuations the plain average */
                    for (int a = 0; a < 3; a++) Sh[3 * i + a] = sp->lsf ? m[a] : m[a] / nn;
                }
            }
        }
        /* A: half drift */
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) pos[3 * i + a] += 0.5 * dt * vel[3 * i + a];
        wrap(n, pos, box, pbc);
        /* full evaluation at (R^{n+1}, S^{n+1}) */
        ctx_init(&C, n, type, pos, spin, box, pbc, params, sp->rcR, sp->rcA, sp->act, use_cells);
        if (sp->zbl[3] > 0) C.zbl = sp->zbl;
        if (sp->landau[0] != 0 || sp->landau[1] != 0) C.landau = sp->landau;
        double E = forward_all(&C, q, Fp, Ei);
        forces_fields(&C, Fp, sp->mu_s, B, F, H);
        double Ez = zeeman(&C, sp->mu_s, B);
        ctx_free(&C);
        /* B: half kick */
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) vel[3 * i + a] += 0.5 * dt * KAPPA * F[3 * i + a] / mt[type[i]];
        *step = st + 1;
        if (obs) {
            or_obs *o = obs + it;
            double ek = 0, num = 0, den = 0, M[3] = {0, 0, 0};
            int nfe = 0;
            for (int i = 0; i < n; i++) {
                ek += 0.5 * mt[type[i]] * dot3(vel + 3 * i, vel + 3 * i) / KAPPA;
                if (type[i] == 0) {
                    double sxh[3];
                    cross3(spin + 3 * i, H + 3 * i, sxh);
                    num += dot3(sxh, sxh);
                    den += dot3(spin + 3 * i, H + 3 * i);
                    for (int a = 0; a < 3; a++) M[a] += spin[3 * i + a];
                    nfe++;
                }
            }
            o->step = (double)(st + 1);
            o->E_nep = E;
            o->E_kin = ek;
            o->E_z = Ez;
            o->T_lat = 2.0 * ek / (3.0 * n * KB);
            o->T_spin = den != 0 ? num / (2.0 * KB * den) : 0.0;
            for (int a = 0; a < 3; a++) o->M[a] = nfe ? M[a] / nfe : 0.0;
            o->passes = passes;
            o->change = change;
            o->capped = capped;
            double sl = 0;
            for (int i = 0; i < n; i++)
                if (type[i] == 0) sl += sqrt(dot3(spin + 3 * i, spin + 3 * i));
            o->s_len = nfe ? sl / nfe : 0.0;
        }
    }
    free(q); free(Fp); free(Ei); free(F); free(H); free(Sn); free(Sh); free(eta); free(snew);
    free(X); free(fk); free(gk); free(fprev); free(gprev); free(xnew); free(dF); free(dG); free(cap_of);
    return 0;
}

/* Field of the frozen-Fp magnetic energy: Fp* from (R, S_hat), evaluated at
 * spins S, plus the Zeeman field; zero rows on non-magnetic atoms. */
int or_field_lin(int n, const int *type, const double *pos, const double *S_hat, const double *S,
                 const double *box, const int *pbc, const double *params, double rcR, double rcA,
                 int act, double mu_s, const double *B, double *H) {
    ctx_t C;
    ctx_init(&C, n, type, pos, S_hat, box, pbc, params, rcR, rcA, act, n > 4096);
    double *q = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Fp = malloc(sizeof(double) * ND * (size_t)(n + 1));
    double *Ei = malloc(sizeof(double) * (n + 1));
    forward_all(&C, q, Fp, Ei);
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) C.spin[3 * i + a] = type[i] == 0 ? S[3 * i + a] : 0.0;
    env_cache(&C);
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; i++) {
        if (type[i] != 0) { H[3 * i] = H[3 * i + 1] = H[3 * i + 2] = 0.0; continue; }
        double hf[3], hs[3];
        hlin_fixed(&C, Fp, i, hf);
        hlin_self(&C, Fp, i, C.spin + 3 * i, hs);
        for (int a = 0; a < 3; a++) H[3 * i + a] = hf[a] + hs[a] + mu_s * MUB * B[a];
    }
    free(q); free(Fp); free(Ei);
    ctx_free(&C);
    return 0;
}
