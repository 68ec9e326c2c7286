/*
 * oracle.c -- plain FP64 CPU oracle of the charge-transfer bond-order
 * potential's energy, forces and charges.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library; the two meet only through the flat
 * parameter vector and the seeded structure generators.
 *
 * What it computes, and where each part comes from:
 *  - neighbours: every (j, image n) with |x_j + n.h - x_i| < cutoff, by brute
 *    force over all atoms and images, or (for large inputs) by a separately
 *    written cell list; self images (j == i, n != 0) are neighbours too;
 *  - energy, forces and the charge solve: oracle_core.h (bond order from the
 *    paper's Methods section, Eqs. 1-7; charges minimise the energy at fixed
 *    total charge, Methods);
 *  - velocity-Verlet NVE dynamics with fixed atoms (the paper fixes the
 *    bottom of its SiC slab while the rest moves);
 *  - parameter derivatives by complex-step differentiation of the same core.
 *
 * Units: Angstrom, eV, e, fs, amu.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* geometry (always real)                                                    */
/* ------------------------------------------------------------------------- */

typedef struct { int j; double d[3]; double r; } pr_t;   /* neighbour entry */
/* CSR over rows; row k is atom rows[k] (rows == NULL: row k is atom k) */
typedef struct { int n; long *off; pr_t *p; int *rows; } nlist_t;

typedef struct {
    double h[3][3];      /* rows: cell vectors */
    double hi[3][3];     /* inverse: frac = x . hi */
    double w[3];         /* perpendicular widths */
    int pbc[3];
} cell_t;

static void cell_init(cell_t *c, const double *box, const int *pbc)
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) c->h[a][b] = box[3 * a + b];
    double (*h)[3] = c->h;
    double det = h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[2][1])
               - h[0][1] * (h[1][0] * h[2][2] - h[1][2] * h[2][0])
               + h[0][2] * (h[1][0] * h[2][1] - h[1][1] * h[2][0]);
    /* inverse of h (frac = x . hi, i.e. x = frac . h) */
    c->hi[0][0] = (h[1][1] * h[2][2] - h[1][2] * h[2][1]) / det;
    c->hi[0][1] = (h[0][2] * h[2][1] - h[0][1] * h[2][2]) / det;
    c->hi[0][2] = (h[0][1] * h[1][2] - h[0][2] * h[1][1]) / det;
    c->hi[1][0] = (h[1][2] * h[2][0] - h[1][0] * h[2][2]) / det;
    c->hi[1][1] = (h[0][0] * h[2][2] - h[0][2] * h[2][0]) / det;
    c->hi[1][2] = (h[0][2] * h[1][0] - h[0][0] * h[1][2]) / det;
    c->hi[2][0] = (h[1][0] * h[2][1] - h[1][1] * h[2][0]) / det;
    c->hi[2][1] = (h[0][1] * h[2][0] - h[0][0] * h[2][1]) / det;
    c->hi[2][2] = (h[0][0] * h[1][1] - h[0][1] * h[1][0]) / det;
    for (int a = 0; a < 3; a++) {
        const double *u = h[(a + 1) % 3], *v = h[(a + 2) % 3];
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        c->w[a] = fabs(det) / sqrt(cx * cx + cy * cy + cz * cz);
        c->pbc[a] = pbc[a] ? 1 : 0;
    }
}

static void to_frac(const cell_t *c, const double *x, double *s)
{
    for (int b = 0; b < 3; b++) s[b] = x[0] * c->hi[0][b] + x[1] * c->hi[1][b] + x[2] * c->hi[2][b];
}

static void to_cart(const cell_t *c, const double *s, double *x)
{
    for (int b = 0; b < 3; b++) x[b] = s[0] * c->h[0][b] + s[1] * c->h[1][b] + s[2] * c->h[2][b];
}

/* positions folded into the cell along periodic vectors */
static double *wrapped(const cell_t *c, int n, const double *pos)
{
    double *xw = malloc(sizeof(double) * 3 * n);
    for (int i = 0; i < n; i++) {
        double s[3];
        to_frac(c, pos + 3 * i, s);
        for (int a = 0; a < 3; a++) if (c->pbc[a]) s[a] -= floor(s[a]);
        to_cart(c, s, xw + 3 * i);
    }
    return xw;
}

static void nl_free(nlist_t *L)
{
    free(L->off);
    free(L->p);
    free(L->rows);
    L->off = NULL;
    L->p = NULL;
    L->rows = NULL;
}

/* Brute force: all atoms j and all images n with |n_a| <= ceil(rc/w_a) + 1
 * along periodic vectors.  Two passes (count, fill) so rows are independent. */
static void nl_brute(const cell_t *c, int n, const double *pos, double rc, nlist_t *L)
{
    double *xw = wrapped(c, n, pos);
    int M[3];
    for (int a = 0; a < 3; a++) M[a] = c->pbc[a] ? (int)ceil(rc / c->w[a]) + 1 : 0;
    L->n = n;
    L->rows = NULL;
    L->off = calloc(n + 1, sizeof(long));
    long *cnt = calloc(n, sizeof(long));
    const double rc2 = rc * rc;
    for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; i++) {
            long k = pass ? L->off[i] : 0;
            for (int j = 0; j < n; j++)
                for (int n0 = -M[0]; n0 <= M[0]; n0++)
                    for (int n1 = -M[1]; n1 <= M[1]; n1++)
                        for (int n2 = -M[2]; n2 <= M[2]; n2++) {
                            if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                            double d[3];
                            for (int a = 0; a < 3; a++)
                                d[a] = xw[3 * j + a] + n0 * c->h[0][a] + n1 * c->h[1][a] + n2 * c->h[2][a] - xw[3 * i + a];
                            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                            if (r2 >= rc2) continue;
                            if (pass) {
                                pr_t *e = &L->p[k];
                                e->j = j;
                                memcpy(e->d, d, sizeof d);
                                e->r = sqrt(r2);
                            }
                            k++;
                        }
            if (!pass) cnt[i] = k;
        }
        if (!pass) {
            for (int i = 0; i < n; i++) L->off[i + 1] = L->off[i] + cnt[i];
            L->p = malloc(sizeof(pr_t) * (L->off[n] > 0 ? L->off[n] : 1));
        }
    }
    free(cnt);
    free(xw);
}

/* Cell list with cells at least rc wide and a +-1 stencil.  Needs >= 3 cells
 * along every periodic vector (returns -1 otherwise).  Along non-periodic
 * vectors the cells span the atoms' range.  With sel != NULL, rows are built
 * only for the nsel atoms listed in sel. */
static int nl_cells_sel(const cell_t *c, int n, const double *pos, double rc, nlist_t *L, const int *sel, int nsel)
{
    double *xw = wrapped(c, n, pos);
    double *s = malloc(sizeof(double) * 3 * n);
    for (int i = 0; i < n; i++) to_frac(c, xw + 3 * i, s + 3 * i);
    double lo[3], hi[3];
    int nb[3];
    for (int a = 0; a < 3; a++) {
        if (c->pbc[a]) {
            lo[a] = 0.0; hi[a] = 1.0;
            nb[a] = (int)floor(c->w[a] / rc);
            if (nb[a] < 3) { free(s); free(xw); return -1; }
        } else {
            lo[a] = 1e300; hi[a] = -1e300;
            for (int i = 0; i < n; i++) { lo[a] = fmin(lo[a], s[3 * i + a]); hi[a] = fmax(hi[a], s[3 * i + a]); }
            double ext = (hi[a] - lo[a]) * c->w[a];
            nb[a] = (int)floor(ext / rc);
            if (nb[a] < 1) nb[a] = 1;
            hi[a] = lo[a] + fmax(hi[a] - lo[a], 1e-12);
        }
    }
    long ncell = (long)nb[0] * nb[1] * nb[2];
    int *cid = malloc(sizeof(int) * n);
    long *head = calloc(ncell + 1, sizeof(long));
    for (int i = 0; i < n; i++) {
        int ci[3];
        for (int a = 0; a < 3; a++) {
            int v = (int)floor((s[3 * i + a] - lo[a]) / (hi[a] - lo[a]) * nb[a]);
            ci[a] = v < 0 ? 0 : (v >= nb[a] ? nb[a] - 1 : v);
        }
        cid[i] = (ci[0] * nb[1] + ci[1]) * nb[2] + ci[2];
        head[cid[i] + 1]++;
    }
    for (long k = 0; k < ncell; k++) head[k + 1] += head[k];
    int *members = malloc(sizeof(int) * n);
    long *fill = calloc((size_t)ncell + 1, sizeof(long));
    for (int i = 0; i < n; i++) members[head[cid[i]] + fill[cid[i]]++] = i;
    free(fill);

    const int nrow = sel ? nsel : n;
    L->n = nrow;
    L->rows = NULL;
    if (sel) {
        L->rows = malloc(sizeof(int) * (nrow > 0 ? nrow : 1));
        memcpy(L->rows, sel, sizeof(int) * nrow);
    }
    L->off = calloc(nrow + 1, sizeof(long));
    long *cnt = calloc(nrow > 0 ? nrow : 1, sizeof(long));
    const double rc2 = rc * rc;
    for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int row = 0; row < nrow; row++) {
            const int i = sel ? sel[row] : row;
            long k = pass ? L->off[row] : 0;
            int c0 = cid[i] / (nb[1] * nb[2]), c1 = (cid[i] / nb[2]) % nb[1], c2 = cid[i] % nb[2];
            for (int d0 = -1; d0 <= 1; d0++)
                for (int d1 = -1; d1 <= 1; d1++)
                    for (int d2 = -1; d2 <= 1; d2++) {
                        int cc[3] = {c0 + d0, c1 + d1, c2 + d2}, im[3] = {0, 0, 0}, skip = 0;
                        for (int a = 0; a < 3; a++) {
                            if (cc[a] < 0 || cc[a] >= nb[a]) {
                                if (!c->pbc[a]) { skip = 1; break; }
                                im[a] = cc[a] < 0 ? -1 : 1;
                                cc[a] -= im[a] * nb[a];
                            }
                        }
                        if (skip) continue;
                        long cell = ((long)cc[0] * nb[1] + cc[1]) * nb[2] + cc[2];
                        for (long m = head[cell]; m < head[cell + 1]; m++) {
                            int j = members[m];
                            if (j == i && im[0] == 0 && im[1] == 0 && im[2] == 0) continue;
                            double d[3];
                            for (int a = 0; a < 3; a++)
                                d[a] = xw[3 * j + a] + im[0] * c->h[0][a] + im[1] * c->h[1][a] + im[2] * c->h[2][a] - xw[3 * i + a];
                            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                            if (r2 >= rc2) continue;
                            if (pass) {
                                pr_t *e = &L->p[k];
                                e->j = j;
                                memcpy(e->d, d, sizeof d);
                                e->r = sqrt(r2);
                            }
                            k++;
                        }
                    }
            if (!pass) cnt[row] = k;
        }
        if (!pass) {
            for (int r = 0; r < nrow; r++) L->off[r + 1] = L->off[r] + cnt[r];
            L->p = malloc(sizeof(pr_t) * (L->off[nrow] > 0 ? L->off[nrow] : 1));
        }
    }
    free(cnt); free(members); free(head); free(cid); free(s); free(xw);
    return 0;
}

static int nl_cells(const cell_t *c, int n, const double *pos, double rc, nlist_t *L)
{
    return nl_cells_sel(c, n, pos, rc, L, NULL, 0);
}

/* method: 0 = brute force, 1 = cell list, -1 = cell list when it applies and
 * n > 2000, brute force otherwise */
static void nl_build(const cell_t *c, int n, const double *pos, double rc, int method, nlist_t *L)
{
    if (method == 1 || (method < 0 && n > 2000)) {
        if (nl_cells(c, n, pos, rc, L) == 0) return;
    }
    nl_brute(c, n, pos, rc, L);
}

/* sub-list of entries with r < rc2 (the short list from the long one) */
static void nl_filter(const nlist_t *A, double rc, nlist_t *B)
{
    int n = A->n;
    B->n = n;
    B->rows = NULL;
    if (A->rows) {
        B->rows = malloc(sizeof(int) * (n > 0 ? n : 1));
        memcpy(B->rows, A->rows, sizeof(int) * n);
    }
    B->off = calloc(n + 1, sizeof(long));
    for (int i = 0; i < n; i++) {
        long k = 0;
        for (long e = A->off[i]; e < A->off[i + 1]; e++) if (A->p[e].r < rc) k++;
        B->off[i + 1] = B->off[i] + k;
    }
    B->p = malloc(sizeof(pr_t) * (B->off[n] > 0 ? B->off[n] : 1));
    for (int i = 0; i < n; i++) {
        long k = B->off[i];
        for (long e = A->off[i]; e < A->off[i + 1]; e++) if (A->p[e].r < rc) B->p[k++] = A->p[e];
    }
}

/* ------------------------------------------------------------------------- */
/* the scalar-generic core, real and complex                                 */
/* ------------------------------------------------------------------------- */

#define SC double
#define FN(x) x##_r
#define RE(x) (x)
#define IM(x) (0.0)
#define SEXP exp
#define SCOS cos
#define SSIN sin
#define SPOW pow
#define SSQRT sqrt
#include "oracle_core.h"
#undef SC
#undef FN
#undef RE
#undef IM
#undef SEXP
#undef SCOS
#undef SSIN
#undef SPOW
#undef SSQRT

#define OR_COMPLEX 1
#define SC double complex
#define FN(x) x##_c
#define RE(x) creal(x)
#define IM(x) cimag(x)
#define SEXP cexp
#define SCOS ccos
#define SSIN csin
#define SPOW cpow
#define SSQRT csqrt
#include "oracle_core.h"

/* ------------------------------------------------------------------------- */
/* exported entry points                                                     */
/* ------------------------------------------------------------------------- */

static double short_cut(const prm_t_r *P)
{
    double s = 0.0;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) s = fmax(s, sqrt(P->sp[a].S * P->sp[b].S));
    return s;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Full evaluation.  pos: n x 3 (row-major), box: 3 x 3 rows, pbc[3].
 * q_io: in = initial charges (warm start), out = equilibrated charges.
 * Outputs E (scalar), F (n x 3), eat (per-atom energy, may be NULL).
 * info[0] = CG iterations (-1: not converged), info[1] = final RMS projected
 * residual, info[2] = mu, info[3] = long-list entries, info[4] = short entries. */
int oracle_eval(int n, const double *pos, const int *types, const double *box, const int *pbc,
                const double *params, double Q, double tol, int maxit, int method,
                double *q_io, double *E, double *F, double *eat, double *info)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t Ll, Ls;
    nl_build(&c, n, pos, P.rc, method, &Ll);
    nl_filter(&Ll, short_cut(&P), &Ls);
    double *Hv = malloc(sizeof(double) * (Ll.off[n] > 0 ? Ll.off[n] : 1));
    assemble_r(&P, n, types, &Ll, Hv);
    double res = 0.0, mu = 0.0;
    int it = qeq_solve_r(&P, n, types, &Ll, Hv, Q, tol, maxit, 0.0, q_io, &res, &mu);
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    double *ea = calloc(n, sizeof(double));
    double Ec = covalent_r(&P, n, types, &Ls, ea, F);
    double Eq = charge_terms_r(&P, n, types, &Ll, q_io, ea, F);
    *E = Ec + Eq;
    if (eat) memcpy(eat, ea, sizeof(double) * n);
    if (info) {
        info[0] = it; info[1] = res; info[2] = mu;
        info[3] = (double)Ll.off[n]; info[4] = (double)Ls.off[n];
    }
    free(ea); free(Hv);
    nl_free(&Ll); nl_free(&Ls);
    return it >= 0 ? 0 : 1;
}

/* Energy and forces at given charges (no charge solve). */
int oracle_eval_fixed_q(int n, const double *pos, const int *types, const double *box, const int *pbc,
                        const double *params, const double *q, int method, double *E, double *F,
                        double *eat)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t Ll, Ls;
    nl_build(&c, n, pos, P.rc, method, &Ll);
    nl_filter(&Ll, short_cut(&P), &Ls);
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    double *ea = calloc(n, sizeof(double));
    double Ec = covalent_r(&P, n, types, &Ls, ea, F);
    double Eq = charge_terms_r(&P, n, types, &Ll, q, ea, F);
    *E = Ec + Eq;
    if (eat) memcpy(eat, ea, sizeof(double) * n);
    free(ea);
    nl_free(&Ll); nl_free(&Ls);
    return 0;
}

/* Dense charge-equilibration matrix H (n x n, row-major) and chi (n): for the
 * direct KKT solve and eigenvalue checks on small inputs. */
int oracle_dense_h(int n, const double *pos, const int *types, const double *box, const int *pbc,
                   const double *params, double *H, double *chi)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t L;
    nl_brute(&c, n, pos, P.rc, &L);
    memset(H, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; i++) {
        H[(long)i * n + i] += P.sp[types[i]].J;
        chi[i] = P.sp[types[i]].chi;
        for (long e = L.off[i]; e < L.off[i + 1]; e++)
            H[(long)i * n + L.p[e].j] += coul_r(&P, types[i], types[L.p[e].j], L.p[e].r, NULL);
    }
    nl_free(&L);
    return 0;
}

/* Bond order of species t for given zeta_1, zeta_2 (and its derivatives). */
double oracle_bond_order(const double *params, int t, double z1, double z2, double *db)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    double z[2] = {z1, z2}, d[2];
    double b = bond_order_r(&P.sp[t], P.p, z, d);
    if (db) { db[0] = d[0]; db[1] = d[1]; }
    return b;
}

/* Angular function w_l of species t at cos(theta). */
double oracle_angular(const double *params, int t, int l, double cs)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    return wang_r(&P.sp[t], l, cs);
}

/* Coulomb kernel C_ij(r) and its derivative. */
double oracle_coulomb(const double *params, int ti, int tj, double r, double *dC)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    return coul_r(&P, ti, tj, r, dC);
}

/* Neighbour list export: counts[n] and, if js != NULL, for every entry the
 * neighbour index and its displacement vector (rows in CSR order). */
long oracle_neighbors(int n, const double *pos, const double *box, const int *pbc, double rc,
                      int method, long *counts, int *js, double *dvec)
{
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t L;
    nl_build(&c, n, pos, rc, method, &L);
    long tot = L.off[n];
    for (int i = 0; i < n; i++) counts[i] = L.off[i + 1] - L.off[i];
    if (js)
        for (long e = 0; e < tot; e++) {
            js[e] = L.p[e].j;
            memcpy(dvec + 3 * e, L.p[e].d, 3 * sizeof(double));
        }
    nl_free(&L);
    return tot;
}

/* Per-atom quantities for a sample of atoms, given charges q for every atom
 * (e.g. a GPU solution), without solving for the charges:
 *   g[s]    = chi_i + (H q)_i   (the charge-equilibration gradient; at the
 *             solution every entry equals mu)
 *   Fs[3s]  = force on atom i (covalent + Coulomb at the given charges)
 *   es[s]   = per-atom energy share of atom i
 * The covalent force on i is taken from a cluster of all atoms within twice
 * the covalent cutoff of i (every term that moves with x_i lies inside it). */
int oracle_sample(int n, const double *pos, const int *types, const double *box, const int *pbc,
                  const double *params, const double *q, int ns, const int *idx,
                  double *g, double *Fs, double *es)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    const double rs = short_cut(&P);
    const double rclu = fmax(P.rc, 2.0 * rs + 1e-6);
    nlist_t L;
    /* rows only for the sampled atoms (cell list), or all rows (brute force) */
    int *rowof = malloc(sizeof(int) * (ns > 0 ? ns : 1));
    if (nl_cells_sel(&c, n, pos, rclu, &L, idx, ns) == 0) {
        for (int s = 0; s < ns; s++) rowof[s] = s;
    } else {
        nl_brute(&c, n, pos, rclu, &L);
        for (int s = 0; s < ns; s++) rowof[s] = idx[s];
    }
    for (int s = 0; s < ns; s++) {
        int i = idx[s], row = rowof[s];
        const sp_t_r *si = &P.sp[types[i]];
        double gi = si->chi + si->J * q[i], f[3] = {0, 0, 0};
        double ei = si->E0 + si->chi * q[i] + 0.5 * si->J * q[i] * q[i];
        int m = 1;
        for (long e = L.off[row]; e < L.off[row + 1]; e++) {
            const pr_t *p = &L.p[e];
            if (p->r < P.rc) {
                double dC, Cv = coul_r(&P, types[i], types[p->j], p->r, &dC);
                gi += Cv * q[p->j];
                ei += 0.5 * q[i] * q[p->j] * Cv;
                if (p->j != i)
                    for (int a = 0; a < 3; a++) f[a] += q[i] * q[p->j] * dC * p->d[a] / p->r;
            }
            if (p->r < 2.0 * rs + 1e-6) m++;
        }
        /* local cluster: atom i at the origin plus every image within 2 rs */
        double *cp = malloc(sizeof(double) * 3 * m);
        int *ct = malloc(sizeof(int) * m);
        cp[0] = cp[1] = cp[2] = 0.0;
        ct[0] = types[i];
        int k = 1;
        for (long e = L.off[row]; e < L.off[row + 1]; e++)
            if (L.p[e].r < 2.0 * rs + 1e-6) {
                memcpy(cp + 3 * k, L.p[e].d, 3 * sizeof(double));
                ct[k++] = types[L.p[e].j];
            }
        double bx[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        int nop[3] = {0, 0, 0};
        cell_t cc;
        cell_init(&cc, bx, nop);
        nlist_t Lc;
        nl_brute(&cc, m, cp, rs, &Lc);
        double *Fc = calloc(3 * m, sizeof(double));
        double *ea = calloc(m, sizeof(double));
        covalent_r(&P, m, ct, &Lc, ea, Fc);
        if (g) g[s] = gi;
        if (Fs) for (int a = 0; a < 3; a++) Fs[3 * s + a] = f[a] + Fc[a];
        if (es) es[s] = ei + ea[0];
        free(ea); free(Fc); free(cp); free(ct);
        nl_free(&Lc);
    }
    free(rowof);
    nl_free(&L);
    return 0;
}

/* Total energy at given charges, streamed over chunks of atoms so the long
 * list never exists whole (for inputs too large for oracle_eval's memory). */
double oracle_energy_at_q(int n, const double *pos, const int *types, const double *box,
                          const int *pbc, const double *params, const double *q, double *eat)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    double *ea = calloc(n, sizeof(double));
    const int chunk = 65536;
    int *sel = malloc(sizeof(int) * chunk);
    for (int a = 0; a < n; a += chunk) {
        int m = (n - a < chunk) ? n - a : chunk;
        for (int k = 0; k < m; k++) sel[k] = a + k;
        nlist_t Ll, Ls;
        if (nl_cells_sel(&c, n, pos, P.rc, &Ll, sel, m) != 0) {
            /* small periodic cell: whole brute-force list */
            nl_brute(&c, n, pos, P.rc, &Ll);
            nl_filter(&Ll, short_cut(&P), &Ls);
            covalent_r(&P, n, types, &Ls, ea, NULL);
            charge_terms_r(&P, n, types, &Ll, q, ea, NULL);
            nl_free(&Ll); nl_free(&Ls);
            break;
        }
        nl_filter(&Ll, short_cut(&P), &Ls);
        double *tmp = calloc(n, sizeof(double));
        covalent_r(&P, n, types, &Ls, tmp, NULL);
        for (int k = 0; k < m; k++) ea[a + k] = tmp[a + k];
        free(tmp);
        charge_terms_r(&P, n, types, &Ll, q, ea, NULL);
        nl_free(&Ll); nl_free(&Ls);
    }
    free(sel);
    double E = 0.0;
    for (int i = 0; i < n; i++) E += ea[i];
    if (eat) memcpy(eat, ea, sizeof(double) * n);
    free(ea);
    return E;
}

/* ------------------------------------------------------------------------- */
/* charge-dependent covalent coupling (stand-in f_q)                         */
/* ------------------------------------------------------------------------- */

/* The paper's potential gives its covalent bonds a covalent-ionic mixed
 * nature through a charge function f_q (Methods, first paragraph) whose form
 * it leaves to its predecessor.  Stand-in: the attraction of bond (i,j) is
 * scaled by f_q = exp(-kappa (q_i - q_j)^2), so the energy is
 *   E(x, q) = E_0(x, q) - 1/2 sum_(i,j) c_ij [f_q(q_i - q_j) - 1],
 *   c_ij = fc(r_ij) b_ij fA(r_ij)   (charge-free attraction of the bond),
 * with E_0 the energy without the coupling.  E is no longer quadratic in q;
 * the charges still minimise it at fixed total charge, found by a nonlinear
 * conjugate-gradient minimisation (Methods: the energy is minimised over the
 * charges by conjugate gradients at every step). */
static double fq_d1(double k, double d) { return -2.0 * k * d * exp(-k * d * d); }
static double fq_d2(double k, double d) { return (4.0 * k * k * d * d - 2.0 * k) * exp(-k * d * d); }

/* dE_c/dq added into g:  E_c = -1/2 sum_e c_e [f_q(q_i - q_j) - 1] over the
 * ordered bonds e = (i,j) of the short list (rows = atoms) */
static void fq_grad(int n, const nlist_t *Ls, const double *cb, double k, const double *q, double *g)
{
    for (int i = 0; i < n; i++)
        for (long e = Ls->off[i]; e < Ls->off[i + 1]; e++) {
            if (cb[e] == 0.0) continue;
            const int j = Ls->p[e].j;
            const double t = -0.5 * cb[e] * fq_d1(k, q[i] - q[j]);
            g[i] += t;
            g[j] -= t;
        }
}

/* the full charge gradient chi + H q + dE_c/dq; hq receives chi + H q */
static void fq_gradient(const prm_t_r *P, int n, const int *types, const nlist_t *Ll, const double *Hv,
                        const nlist_t *Ls, const double *cb, double k, const double *q, double *hq, double *g)
{
    matvec_r(P, n, types, Ll, Hv, q, hq);
    for (int i = 0; i < n; i++) {
        hq[i] += P->sp[types[i]].chi;
        g[i] = hq[i];
    }
    fq_grad(n, Ls, cb, k, q, g);
}

/* z = D^-1 (r - w 1) with w such that sum z = 0 (the projected Jacobi step).
 * r is shifted by w in place: since sum z = 0 no dot product with z changes,
 * and r then carries no large constant part (the multiplier mu) whose
 * rounding would swamp those products near convergence. */
static void fq_precond(int n, const double *dinv, double sdinv, double *r, double *z)
{
    double srd = 0.0;
    for (int i = 0; i < n; i++) srd += r[i] * dinv[i];
    const double w = srd / sdinv;
    for (int i = 0; i < n; i++) {
        r[i] -= w;
        z[i] = dinv[i] * r[i];
    }
}

/* Minimise E over q with sum q = Q by projected, Jacobi-preconditioned
 * nonlinear conjugate gradients (Polak-Ribiere with restart at beta < 0).
 * The step length along each direction p minimises E(q + a p) by Newton's
 * method on phi'(a) = p.g(q) + a p.H p + p.[dE_c/dq(q + a p) - dE_c/dq(q)], with
 * phi''(a) = p.H p - 1/2 sum_e c_e f_q''(.) (p_i - p_j)^2.  Every gradient is
 * recomputed from its definition, so nothing drifts.  Stops when the RMS of
 * the projected gradient is below tol.  Returns the iteration count, -1 if
 * maxit was reached, -2 if the energy is not convex along a direction. */
static int fq_solve(const prm_t_r *P, int n, const int *types, const nlist_t *Ll, const double *Hv,
                    const nlist_t *Ls, const double *cb, double k, double Q, double tol, int maxit,
                    double *q, double *res_out, double *mu_out)
{
    double *dinv = calloc(n, sizeof(double)), *hq = calloc(n, sizeof(double)), *g = calloc(n, sizeof(double));
    double *r = calloc(n, sizeof(double)), *z = calloc(n, sizeof(double)), *p = calloc(n, sizeof(double));
    double *s = calloc(n, sizeof(double)), *qa = calloc(n, sizeof(double)), *ga = calloc(n, sizeof(double));
    double sdinv = 0.0;
    for (int i = 0; i < n; i++) {
        double d = P->sp[types[i]].J;
        for (long e = Ll->off[i]; e < Ll->off[i + 1]; e++)
            if (Ll->p[e].j == i) d += Hv[e];
        dinv[i] = 1.0 / d;
        sdinv += dinv[i];
    }
    double sq = 0.0;
    for (int i = 0; i < n; i++) sq += q[i];
    for (int i = 0; i < n; i++) q[i] += (Q - sq) / n;
    fq_gradient(P, n, types, Ll, Hv, Ls, cb, k, q, hq, g);
    for (int i = 0; i < n; i++) r[i] = -g[i];
    fq_precond(n, dinv, sdinv, r, z);
    double rz = 0.0;
    for (int i = 0; i < n; i++) { p[i] = z[i]; rz += r[i] * z[i]; }
    int it = 0, rc = -1;
    double res = 0.0;
    for (;;) {
        double sr = 0.0, nr = 0.0;
        for (int i = 0; i < n; i++) sr += r[i];
        for (int i = 0; i < n; i++) nr += (r[i] - sr / n) * (r[i] - sr / n);
        res = sqrt(nr / n);
        if (res < tol) { rc = it; break; }
        if (it >= maxit) break;
        matvec_r(P, n, types, Ll, Hv, p, s);
        /* phi'(0) = p.g = -p.r with the shifted r (p.(chi + H q) directly
         * would cancel the multiplier's share in rounding) */
        double pHp = 0.0, pr = 0.0, pg0c = 0.0;
        for (int i = 0; i < n; i++) { pHp += p[i] * s[i]; pr += p[i] * r[i]; }
        if (!(pHp > 0.0)) { rc = -2; break; }
        for (int i = 0; i < n; i++) ga[i] = 0.0;
        fq_grad(n, Ls, cb, k, q, ga);
        for (int i = 0; i < n; i++) pg0c += p[i] * ga[i];
        /* line search */
        double a = 0.0;
        int convex = 1;
        for (int ls = 0; ls < 60; ls++) {
            for (int i = 0; i < n; i++) { qa[i] = q[i] + a * p[i]; ga[i] = 0.0; }
            fq_grad(n, Ls, cb, k, qa, ga);
            double d1 = -pr + a * pHp - pg0c, d2 = pHp;
            for (int i = 0; i < n; i++) d1 += p[i] * ga[i];
            for (int i = 0; i < n; i++)
                for (long e = Ls->off[i]; e < Ls->off[i + 1]; e++) {
                    if (cb[e] == 0.0) continue;
                    const int j = Ls->p[e].j;
                    const double dp = p[i] - p[j];
                    d2 += -0.5 * cb[e] * fq_d2(k, qa[i] - qa[j]) * dp * dp;
                }
            if (!(d2 > 0.0)) { convex = 0; break; }
            const double step = d1 / d2;
            a -= step;
            if (fabs(step) <= 1e-15 * fabs(a)) break;
        }
        if (!convex) { rc = -2; break; }
        for (int i = 0; i < n; i++) q[i] += a * p[i];
        fq_gradient(P, n, types, Ll, Hv, Ls, cb, k, q, hq, g);
        /* new residual and direction (Polak-Ribiere, restarted when negative) */
        double *rn = ga;
        for (int i = 0; i < n; i++) rn[i] = -g[i];
        fq_precond(n, dinv, sdinv, rn, z);
        double num = 0.0, rzn = 0.0;
        for (int i = 0; i < n; i++) { num += z[i] * (rn[i] - r[i]); rzn += z[i] * rn[i]; }
        double beta = num / rz;
        if (beta < 0.0) beta = 0.0;
        for (int i = 0; i < n; i++) { p[i] = z[i] + beta * p[i]; r[i] = rn[i]; }
        rz = rzn;
        it++;
    }
    double sq2 = 0.0;
    for (int i = 0; i < n; i++) sq2 += q[i];
    for (int i = 0; i < n; i++) q[i] += (Q - sq2) / n;
    fq_gradient(P, n, types, Ll, Hv, Ls, cb, k, q, hq, g);
    double mu = 0.0;
    for (int i = 0; i < n; i++) mu += g[i];
    if (mu_out) *mu_out = mu / n;
    if (res_out) *res_out = res;
    free(dinv); free(hq); free(g); free(r); free(z); free(p); free(s); free(qa); free(ga);
    return rc;
}

/* Full evaluation with the charge coupling of strength kappa (arguments and
 * info as for oracle_eval; info[0] = -2 if the energy was not convex in q
 * along a search direction).  kappa = 0 reduces to the quadratic energy. */
int oracle_eval_fq(int n, const double *pos, const int *types, const double *box, const int *pbc,
                   const double *params, double kappa, double Q, double tol, int maxit, int method,
                   double *q_io, double *E, double *F, double *eat, double *info)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t Ll, Ls;
    nl_build(&c, n, pos, P.rc, method, &Ll);
    nl_filter(&Ll, short_cut(&P), &Ls);
    double *Hv = malloc(sizeof(double) * (Ll.off[n] > 0 ? Ll.off[n] : 1));
    double *cb = calloc(Ls.off[n] > 0 ? Ls.off[n] : 1, sizeof(double));
    assemble_r(&P, n, types, &Ll, Hv);
    covalent_q_r(&P, n, types, &Ls, NULL, 0.0, cb, NULL, NULL);      /* c_e only */
    double res = 0.0, mu = 0.0;
    int it = fq_solve(&P, n, types, &Ll, Hv, &Ls, cb, kappa, Q, tol, maxit, q_io, &res, &mu);
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    double *ea = calloc(n, sizeof(double));
    double Ec = covalent_q_r(&P, n, types, &Ls, q_io, kappa, NULL, ea, F);
    double Eq = charge_terms_r(&P, n, types, &Ll, q_io, ea, F);
    *E = Ec + Eq;
    if (eat) memcpy(eat, ea, sizeof(double) * n);
    if (info) {
        info[0] = it; info[1] = res; info[2] = mu;
        info[3] = (double)Ll.off[n]; info[4] = (double)Ls.off[n];
    }
    free(ea); free(Hv); free(cb);
    nl_free(&Ll); nl_free(&Ls);
    return it >= 0 ? 0 : 1;
}

/* Energy, forces and the charge gradient g = dE/dq at given charges q, with
 * the coupling of strength kappa (no charge minimisation). */
int oracle_eval_fq_fixed(int n, const double *pos, const int *types, const double *box, const int *pbc,
                         const double *params, double kappa, const double *q, int method, double *E,
                         double *F, double *g)
{
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t Ll, Ls;
    nl_build(&c, n, pos, P.rc, method, &Ll);
    nl_filter(&Ll, short_cut(&P), &Ls);
    double *Hv = malloc(sizeof(double) * (Ll.off[n] > 0 ? Ll.off[n] : 1));
    double *cb = calloc(Ls.off[n] > 0 ? Ls.off[n] : 1, sizeof(double));
    double *hq = calloc(n, sizeof(double));
    assemble_r(&P, n, types, &Ll, Hv);
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    double Ec = covalent_q_r(&P, n, types, &Ls, q, kappa, cb, NULL, F);
    double Eq = charge_terms_r(&P, n, types, &Ll, q, NULL, F);
    *E = Ec + Eq;
    if (g) fq_gradient(&P, n, types, &Ll, Hv, &Ls, cb, kappa, q, hq, g);
    free(Hv); free(cb); free(hq);
    nl_free(&Ll); nl_free(&Ls);
    return 0;
}

/* Velocity-Verlet NVE: half kick, drift, new forces (charges re-equilibrated,
 * warm-started), half kick.  Fixed atoms (fixed[i] != 0) neither move nor
 * change velocity but still interact.  Velocities in Angstrom/fs.
 * Etraj[s] (s = 0..nsteps) = potential + kinetic energy after step s. */
int oracle_md_nve(int n, double *pos, double *vel, const int *types, const int *fixed,
                  const double *box, const int *pbc, const double *params, double Q, double dt,
                  int nsteps, double tol, double *q_io, double *Etraj, double *Epot)
{
    const double acc = 9.648533212e-3;        /* (eV/Angstrom)/amu in Angstrom/fs^2 */
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    double *F = malloc(sizeof(double) * 3 * n), E;
    double info[5];
    if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
        free(F);
        return 1;
    }
    for (int s = 0; s <= nsteps; s++) {
        if (s > 0) {
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                double m = P.sp[types[i]].mass;
                for (int a = 0; a < 3; a++) {
                    vel[3 * i + a] += 0.5 * dt * acc * F[3 * i + a] / m;
                    pos[3 * i + a] += dt * vel[3 * i + a];
                }
            }
            if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
                free(F);
                return 1;
            }
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                double m = P.sp[types[i]].mass;
                for (int a = 0; a < 3; a++) vel[3 * i + a] += 0.5 * dt * acc * F[3 * i + a] / m;
            }
        }
        double ke = 0.0;
        for (int i = 0; i < n; i++) {
            double m = P.sp[types[i]].mass;
            for (int a = 0; a < 3; a++) ke += 0.5 * m * vel[3 * i + a] * vel[3 * i + a] / acc;
        }
        if (Etraj) Etraj[s] = E + ke;
        if (Epot) Epot[s] = E;
    }
    free(F);
    return 0;
}

/* NVT molecular dynamics with a Nose-Hoover chain thermostat.  The paper runs
 * its growth MD in the NVT ensemble at 2500 K with the bottom of the slab fixed
 * (growth-simulation section) without naming the thermostat; a chain of M
 * Nose-Hoover thermostats is the stated reading.  Equations of motion, with
 * K the kinetic energy of the mobile atoms and Nf their degrees of freedom:
 *   dx/dt = v,   m dv/dt = F - m vxi_1 v,
 *   Q_1 dvxi_1/dt = 2K - Nf kT - Q_1 vxi_1 vxi_2,
 *   Q_k dvxi_k/dt = Q_{k-1} vxi_{k-1}^2 - kT - Q_k vxi_k vxi_{k+1}   (1 < k < M),
 *   Q_M dvxi_M/dt = Q_{M-1} vxi_{M-1}^2 - kT,   dxi_k/dt = vxi_k,
 * with Q_1 = Nf kT tau^2 and Q_k = kT tau^2.  The conserved quantity is
 *   E_pot + K + sum_k Q_k vxi_k^2 / 2 + Nf kT xi_1 + kT sum_{k>1} xi_k.
 * Integration: a thermostat half step, a velocity-Verlet step, a thermostat
 * half step.  The thermostat half step (length h = dt/2) propagates the chain
 * velocities from the last member down to the first (each force G_k applied
 * for h/2 between two damping factors exp(-vxi_{k+1} h/4)), scales the
 * particle velocities by exp(-vxi_1 h), advances xi_k by vxi_k h, and then
 * repeats the chain update from the first member up to the last.  Each piece
 * is an exact flow of part of the equations, so the step is time reversible.
 * Nf = 3 N_mobile, less 3 when no atom is fixed (momentum is then conserved). */
static double nhc_force(int k, int M, double K, double Nf, double kT, const double *Qm, const double *vxi)
{
    (void)M;
    if (k == 0) return (2.0 * K - Nf * kT) / Qm[0];
    return (Qm[k - 1] * vxi[k - 1] * vxi[k - 1] - kT) / Qm[k];
}

static double nhc_half_step(int M, double h, double *K, double Nf, double kT, const double *Qm, double *xi,
                            double *vxi)
{
    /* down the chain */
    vxi[M - 1] += 0.5 * h * nhc_force(M - 1, M, *K, Nf, kT, Qm, vxi);
    for (int k = M - 2; k >= 0; k--) {
        const double damp = exp(-0.25 * h * vxi[k + 1]);
        vxi[k] *= damp;
        vxi[k] += 0.5 * h * nhc_force(k, M, *K, Nf, kT, Qm, vxi);
        vxi[k] *= damp;
    }
    const double scale = exp(-h * vxi[0]);
    *K *= scale * scale;
    for (int k = 0; k < M; k++) xi[k] += h * vxi[k];
    /* up the chain */
    for (int k = 0; k < M - 1; k++) {
        const double damp = exp(-0.25 * h * vxi[k + 1]);
        vxi[k] *= damp;
        vxi[k] += 0.5 * h * nhc_force(k, M, *K, Nf, kT, Qm, vxi);
        vxi[k] *= damp;
    }
    vxi[M - 1] += 0.5 * h * nhc_force(M - 1, M, *K, Nf, kT, Qm, vxi);
    return scale;
}

/* Etraj[s] receives the conserved quantity, Epot[s] the potential energy and
 * Ekin[s] the kinetic energy of the mobile atoms, s = 0..nsteps.  xi, vxi (M
 * each) hold the chain state in and out. */
int oracle_md_nvt(int n, double *pos, double *vel, const int *types, const int *fixed, const double *box,
                  const int *pbc, const double *params, double Q, double dt, int nsteps, double T, double tau,
                  int M, double *xi, double *vxi, double tol, double *q_io, double *Etraj, double *Epot,
                  double *Ekin)
{
    const double acc = 9.648533212e-3;        /* (eV/Angstrom)/amu in Angstrom/fs^2 */
    const double kB = 8.617333262e-5;         /* eV/K */
    if (M < 1 || M > 16) return 2;
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    int nmob = 0;
    for (int i = 0; i < n; i++) nmob += (fixed && fixed[i]) ? 0 : 1;
    const double Nf = 3.0 * nmob - (nmob == n ? 3.0 : 0.0);
    const double kT = kB * T;
    double Qm[16];
    for (int k = 0; k < M; k++) Qm[k] = (k == 0 ? Nf : 1.0) * kT * tau * tau;
    double *F = malloc(sizeof(double) * 3 * n), E;
    double info[5];
    if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
        free(F);
        return 1;
    }
    for (int s = 0; s <= nsteps; s++) {
        if (s > 0) {
            double K = 0.0;
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                const double m = P.sp[types[i]].mass;
                for (int a = 0; a < 3; a++) K += 0.5 * m * vel[3 * i + a] * vel[3 * i + a] / acc;
            }
            double sc = nhc_half_step(M, 0.5 * dt, &K, Nf, kT, Qm, xi, vxi);
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                const double m = P.sp[types[i]].mass;
                for (int a = 0; a < 3; a++) {
                    vel[3 * i + a] = sc * vel[3 * i + a] + 0.5 * dt * acc * F[3 * i + a] / m;
                    pos[3 * i + a] += dt * vel[3 * i + a];
                }
            }
            if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
                free(F);
                return 1;
            }
            K = 0.0;
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                const double m = P.sp[types[i]].mass;
                for (int a = 0; a < 3; a++) {
                    vel[3 * i + a] += 0.5 * dt * acc * F[3 * i + a] / m;
                    K += 0.5 * m * vel[3 * i + a] * vel[3 * i + a] / acc;
                }
            }
            sc = nhc_half_step(M, 0.5 * dt, &K, Nf, kT, Qm, xi, vxi);
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                for (int a = 0; a < 3; a++) vel[3 * i + a] *= sc;
            }
        }
        double K = 0.0, Eth = Nf * kT * xi[0];
        for (int i = 0; i < n; i++) {
            if (fixed && fixed[i]) continue;
            const double m = P.sp[types[i]].mass;
            for (int a = 0; a < 3; a++) K += 0.5 * m * vel[3 * i + a] * vel[3 * i + a] / acc;
        }
        for (int k = 0; k < M; k++) Eth += 0.5 * Qm[k] * vxi[k] * vxi[k] + (k > 0 ? kT * xi[k] : 0.0);
        if (Etraj) Etraj[s] = E + K + Eth;
        if (Epot) Epot[s] = E;
        if (Ekin) Ekin[s] = K;
    }
    free(F);
    return 0;
}

/* Structure relaxation by FIRE (Bitzek, Koskinen, Gaehler, Moseler and
 * Gumbsch, Phys. Rev. Lett. 97, 170201 (2006)).  The paper relaxes its
 * graphene-on-SiC structures and annealed samples without naming the
 * minimiser; FIRE is the stated reading.  Starting from rest with step dt0,
 * mixing alpha_start and a count of uphill-free steps n_pos = 0, each
 * iteration takes one velocity-Verlet step of length dt with the atoms' own
 * masses, stops when the largest force on a mobile atom is below fmax, and
 * otherwise, with P = F.v and norms |v|, |F| over all mobile components:
 *   v <- (1 - alpha) v + alpha |v| F / |F|;
 *   P > 0:  n_pos += 1, and once n_pos > n_min:  dt <- min(f_inc dt, dtmax),
 *           alpha <- f_alpha alpha;
 *   P <= 0: dt <- f_dec dt, v <- 0, alpha <- alpha_start, n_pos <- 0.
 * n_min = 5, f_inc = 1.1, f_dec = 0.5, alpha_start = 0.1, f_alpha = 0.99 (the
 * published values).  Fixed atoms neither move nor enter P, the norms or the
 * convergence test.  Etrace[s] (s = 0..steps, may be NULL; room for
 * max_steps + 1) gets the energy after step s.  Returns 0 and sets *steps
 * (iterations taken), *fmax_out and *converged; 1 if a charge solve fails. */
int oracle_relax_fire(int n, double *pos, const int *types, const int *fixed, const double *box, const int *pbc,
                      const double *params, double Q, double fmax, int max_steps, double dt0, double dtmax,
                      double tol, double *q_io, double *Etrace, int *steps, double *fmax_out, int *converged)
{
    const double acc = 9.648533212e-3;        /* (eV/Angstrom)/amu in Angstrom/fs^2 */
    const int n_min = 5;
    const double f_inc = 1.1, f_dec = 0.5, alpha_start = 0.1, f_alpha = 0.99;
    prm_t_r P;
    read_params_r(params, -1, 0.0, &P);
    double *F = malloc(sizeof(double) * 3 * n), *vel = calloc(3 * n, sizeof(double)), E;
    double info[5];
    double dt = dt0, alpha = alpha_start;
    int n_pos = 0, s = 0;
    *converged = 0;
    if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
        free(F);
        free(vel);
        return 1;
    }
    for (;;) {
        double fm2 = 0.0;
        for (int i = 0; i < n; i++) {
            if (fixed && fixed[i]) continue;
            const double f2 = F[3 * i] * F[3 * i] + F[3 * i + 1] * F[3 * i + 1] + F[3 * i + 2] * F[3 * i + 2];
            if (f2 > fm2) fm2 = f2;
        }
        if (Etrace) Etrace[s] = E;
        *fmax_out = sqrt(fm2);
        if (*fmax_out < fmax) {
            *converged = 1;
            break;
        }
        if (s == max_steps) break;
        if (s > 0) {
            /* F1-F4 on the state after the last MD step */
            double Pw = 0.0, vv = 0.0, ff = 0.0;
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                for (int a = 0; a < 3; a++) {
                    Pw += F[3 * i + a] * vel[3 * i + a];
                    vv += vel[3 * i + a] * vel[3 * i + a];
                    ff += F[3 * i + a] * F[3 * i + a];
                }
            }
            const double c = ff > 0.0 ? alpha * sqrt(vv) / sqrt(ff) : 0.0;
            for (int i = 0; i < n; i++) {
                if (fixed && fixed[i]) continue;
                for (int a = 0; a < 3; a++) vel[3 * i + a] = (1.0 - alpha) * vel[3 * i + a] + c * F[3 * i + a];
            }
            if (Pw > 0.0) {
                n_pos++;
                if (n_pos > n_min) {
                    dt = fmin(dt * f_inc, dtmax);
                    alpha *= f_alpha;
                }
            } else {
                dt *= f_dec;
                for (int k = 0; k < 3 * n; k++) vel[k] = 0.0;
                alpha = alpha_start;
                n_pos = 0;
            }
        }
        /* MD step */
        for (int i = 0; i < n; i++) {
            if (fixed && fixed[i]) continue;
            const double m = P.sp[types[i]].mass;
            for (int a = 0; a < 3; a++) {
                vel[3 * i + a] += 0.5 * dt * acc * F[3 * i + a] / m;
                pos[3 * i + a] += dt * vel[3 * i + a];
            }
        }
        if (oracle_eval(n, pos, types, box, pbc, params, Q, tol, 2000, -1, q_io, &E, F, NULL, info)) {
            free(F);
            free(vel);
            return 1;
        }
        for (int i = 0; i < n; i++) {
            if (fixed && fixed[i]) continue;
            const double m = P.sp[types[i]].mass;
            for (int a = 0; a < 3; a++) vel[3 * i + a] += 0.5 * dt * acc * F[3 * i + a] / m;
        }
        s++;
    }
    *steps = s;
    free(F);
    free(vel);
    return 0;
}

/* Parameter derivatives by complex step: for parameter k, dE/dtheta_k,
 * dF/dtheta_k (n x 3) and dq/dtheta_k (n), all at the equilibrated charges
 * (the charge solve is redone in complex arithmetic, so the charges' response
 * to theta_k is included).  h is the imaginary step (e.g. 1e-30). */
int oracle_param_derivative(int n, const double *pos, const int *types, const double *box,
                            const int *pbc, const double *params, double Q, double tol, int k,
                            double h, double *dE, double *dF, double *dq, double *E, double *F,
                            double *q)
{
    prm_t_c P;
    read_params_c(params, k, h, &P);
    prm_t_r Pr;
    read_params_r(params, -1, 0.0, &Pr);
    cell_t c;
    cell_init(&c, box, pbc);
    nlist_t Ll, Ls;
    nl_build(&c, n, pos, creal(P.rc), -1, &Ll);
    nl_filter(&Ll, short_cut(&Pr), &Ls);
    double complex *Hv = malloc(sizeof(double complex) * (Ll.off[n] > 0 ? Ll.off[n] : 1));
    assemble_c(&P, n, types, &Ll, Hv);
    double complex *qc = calloc(n, sizeof(double complex));
    double res;
    double complex mu;
    int it = qeq_solve_c(&P, n, types, &Ll, Hv, Q, tol, 5000, h, qc, &res, &mu);
    double complex *Fc = calloc(3 * n, sizeof(double complex));
    double complex Ec = covalent_c(&P, n, types, &Ls, NULL, Fc);
    double complex Eq = charge_terms_c(&P, n, types, &Ll, qc, NULL, Fc);
    double complex Et = Ec + Eq;
    if (dE) *dE = cimag(Et) / h;
    if (E) *E = creal(Et);
    for (int i = 0; i < n; i++) {
        if (dq) dq[i] = cimag(qc[i]) / h;
        if (q) q[i] = creal(qc[i]);
        for (int a = 0; a < 3; a++) {
            if (dF) dF[3 * i + a] = cimag(Fc[3 * i + a]) / h;
            if (F) F[3 * i + a] = creal(Fc[3 * i + a]);
        }
    }
    free(Fc); free(qc); free(Hv);
    nl_free(&Ll); nl_free(&Ls);
    return it >= 0 ? 0 : 1;
}
