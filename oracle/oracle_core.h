/*
 * oracle_core.h -- scalar-generic core of the CPU oracle (TEST INFRASTRUCTURE).
 *
 * This file is included twice by oracle.c: once with SC = double and once with
 * SC = double complex.  The complex build evaluates the same definitions with
 * one parameter carrying an imaginary perturbation i*h, so that Im(result)/h is
 * the exact parameter derivative (complex-step differentiation, Squire & Trapp
 * 1998).  Geometry (positions, distances, neighbour lists) is always real; only
 * parameters and everything computed from them take the scalar type SC.  Every
 * branch tests real parts, and every dot product is unconjugated, so each
 * operation is an analytic function of the parameters.
 *
 * What is computed (the energy of the charge-transfer bond-order potential):
 *
 *   E = sum_i [E0_i + chi_i q_i + J_i q_i^2 / 2]                    self energy
 *     + 1/2 sum_i sum_(j,n)!=(i,0) q_i q_j C_ij(r)                    Coulomb
 *     + 1/2 sum_i sum_(j,n) fc(r) [fR(r) - b_ij fA(r)]                covalent
 *
 * The bond order b_ij is the paper's vectorised form (Methods, Eqs. 3-5 and the
 * expanded two-channel Eq. 7, p = 2), normalised by G so that b = 1 when every
 * zeta_l = 0.  zeta_l,ij is a Tersoff-type sum over k (Eq. 2).  The pair terms
 * fR, fA, fc, the angular functions w_l, the self energy (with the constant
 * term E0 of the Methods section) and the shielded, tapered Coulomb kernel are
 * the stand-in functional form, written out where used below.
 *
 * Charges minimise E over q with sum q = Q (Methods: charges are minimised by
 * conjugate gradients at every step).  E is quadratic in q, so the minimiser
 * solves H q + chi = mu 1, 1^T q = Q with H = diag(J) + [C_ij summed over
 * images].  With the optional charge-dependent coupling of the covalent part
 * (covalent_q below) E is no longer quadratic in q; oracle.c minimises it by
 * nonlinear conjugate gradients.
 */

/* ------------------------------------------------------------------------- */
/* parameters                                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    SC A, B, lam1, lam2, R, S, sigma;
    SC gam[2], c[2], d[2], h[2], nn[2], g[2], alpha[2];
    SC chi, J, gc, E0, mass;
    SC G;                       /* normalisation constant, derived */
} FN(sp_t);

typedef struct {
    FN(sp_t) sp[2];
    SC Bmix, ke, rc, p;
} FN(prm_t);

/* Read the flat 56-double layout; parameter `pk` (if >= 0) gets the imaginary
 * perturbation `ph` (complex build only). */
static void FN(read_params)(const double *f, int pk, double ph, FN(prm_t) *P)
{
    SC v[56];
    for (int i = 0; i < 56; i++) v[i] = f[i];
#ifdef OR_COMPLEX
    if (pk >= 0 && pk < 56) v[pk] += I * ph;
#else
    (void)pk; (void)ph;
#endif
    for (int t = 0; t < 2; t++) {
        const SC *s = v + 26 * t;
        FN(sp_t) *q = &P->sp[t];
        q->A = s[0]; q->B = s[1]; q->lam1 = s[2]; q->lam2 = s[3];
        q->R = s[4]; q->S = s[5]; q->sigma = s[6];
        for (int l = 0; l < 2; l++) {
            const SC *c = s + 7 + 7 * l;
            q->gam[l] = c[0]; q->c[l] = c[1]; q->d[l] = c[2]; q->h[l] = c[3];
            q->nn[l] = c[4]; q->g[l] = c[5]; q->alpha[l] = c[6];
        }
        q->chi = s[21]; q->J = s[22]; q->gc = s[23]; q->E0 = s[24]; q->mass = s[25];
    }
    P->Bmix = v[52]; P->ke = v[53]; P->rc = v[54]; P->p = v[55];
    /* G: b = 1 when zeta_1 = zeta_2 = 0 (normalisation stated after Eq. 5 and
     * after Eq. 7):  b(0) = G (g1^-p + g2^-p)^(1/(2 sigma p)) = 1. */
    for (int t = 0; t < 2; t++) {
        FN(sp_t) *q = &P->sp[t];
        SC s0 = SPOW(q->g[0], -P->p) + SPOW(q->g[1], -P->p);
        q->G = SPOW(s0, -1.0 / (2.0 * q->sigma * P->p));
    }
}

/* Pair parameters: A, B geometric means (B scaled by the Si-C factor for
 * unlike pairs), lambdas arithmetic means, cutoffs R, S geometric means. */
typedef struct { SC A, B, lam1, lam2, R, S; } FN(pair_t);

static FN(pair_t) FN(pair_params)(const FN(prm_t) *P, int ti, int tj)
{
    const FN(sp_t) *a = &P->sp[ti], *b = &P->sp[tj];
    FN(pair_t) o;
    o.A = SSQRT(a->A * b->A);
    o.B = SSQRT(a->B * b->B) * (ti != tj ? P->Bmix : 1.0);
    o.lam1 = 0.5 * (a->lam1 + b->lam1);
    o.lam2 = 0.5 * (a->lam2 + b->lam2);
    o.R = SSQRT(a->R * b->R);
    o.S = SSQRT(a->S * b->S);
    return o;
}

/* ------------------------------------------------------------------------- */
/* elementary functions                                                      */
/* ------------------------------------------------------------------------- */

/* smooth cutoff: 1 below R, 0 above S, half-cosine in between */
static SC FN(fc)(double r, SC R, SC S)
{
    if (r <= RE(R)) return 1.0;
    if (r >= RE(S)) return 0.0;
    return 0.5 + 0.5 * SCOS(M_PI * (r - R) / (S - R));
}

static SC FN(dfc)(double r, SC R, SC S)
{
    if (r <= RE(R) || r >= RE(S)) return 0.0;
    return -0.5 * M_PI / (S - R) * SSIN(M_PI * (r - R) / (S - R));
}

/* angular function of channel l of species t, minimal at cos(theta) = h:
 * w = gamma [1 + c^2 x^2 / (d^2 (d^2 + x^2))], x = h - cos(theta) */
static SC FN(wang)(const FN(sp_t) *s, int l, double cs)
{
    SC x = s->h[l] - cs;
    SC c2 = s->c[l] * s->c[l], d2 = s->d[l] * s->d[l];
    return s->gam[l] * (1.0 + c2 * x * x / (d2 * (d2 + x * x)));
}

static SC FN(dwang)(const FN(sp_t) *s, int l, double cs)   /* d w / d cos(theta) */
{
    SC x = s->h[l] - cs;
    SC c2 = s->c[l] * s->c[l], d2 = s->d[l] * s->d[l];
    SC den = d2 + x * x;
    return -s->gam[l] * c2 * 2.0 * x / (den * den);
}

/* radial factor exp[(alpha (r_ij - r_ik))^3] and its derivative in the argument */
static SC FN(eexp)(SC alpha, double dl)
{
    SC a = alpha * dl;
    return SEXP(a * a * a);
}

static SC FN(deexp)(SC alpha, double dl)
{
    SC a = alpha * dl;
    return 3.0 * alpha * a * a * SEXP(a * a * a);
}

/* Vectorised bond order (Eqs. 3-5, 7):
 *   zhat_l = g_l + zeta_l^n_l,  b = G (sum_l zhat_l^-p)^(1/(2 sigma p))
 * and db/dzeta_l = -b n_l zeta_l^(n_l-1) zhat_l^(-p-1) / (2 sigma sum_l zhat_l^-p);
 * the derivative of a channel with zeta_l = 0 is taken as its limit, 0. */
static SC FN(bond_order)(const FN(sp_t) *s, SC p, const SC z[2], SC db[2])
{
    SC zh[2], zn[2], sum = 0.0;
    for (int l = 0; l < 2; l++) {
        zn[l] = (RE(z[l]) > 0.0) ? SPOW(z[l], s->nn[l]) : 0.0;
        zh[l] = s->g[l] + zn[l];
        sum += SPOW(zh[l], -p);
    }
    SC b = s->G * SPOW(sum, 1.0 / (2.0 * s->sigma * p));
    for (int l = 0; l < 2; l++) {
        if (RE(z[l]) > 0.0)
            db[l] = -b * s->nn[l] * (zn[l] / z[l]) * SPOW(zh[l], -p - 1.0) / (2.0 * s->sigma * sum);
        else
            db[l] = 0.0;
    }
    return b;
}

/* Shielded, tapered Coulomb kernel
 *   C(r) = ke T(r/rc) (r^3 + gamma_ij^-3)^(-1/3),  gamma_ij = sqrt(gamma_i gamma_j)
 *   T(x) = 1 - 35x^4 + 84x^5 - 70x^6 + 20x^7 (x < 1), 0 beyond. */
static SC FN(coul)(const FN(prm_t) *P, int ti, int tj, double r, SC *dC)
{
    if (r >= RE(P->rc)) { if (dC) *dC = 0.0; return 0.0; }
    SC x = r / P->rc;
    SC x2 = x * x, x3 = x2 * x;
    SC om = 1.0 - x, om2 = om * om;
    /* the same polynomial written as (1-x)^4 (1 + 4x + 10x^2 + 20x^3), which
     * has no cancellation near the cutoff */
    SC T = om2 * om2 * (1.0 + 4.0 * x + 10.0 * x2 + 20.0 * x3);
    SC dT = -140.0 * x3 * om2 * om;
    SC g3 = SPOW(P->sp[ti].gc * P->sp[tj].gc, -1.5);      /* gamma_ij^-3 */
    SC u = r * r * r + g3;
    SC s = SPOW(u, -1.0 / 3.0);
    if (dC) *dC = P->ke * (dT / P->rc * s - T * r * r * s * s * s * s);
    return P->ke * T * s;
}

/* ------------------------------------------------------------------------- */
/* covalent energy and forces                                                */
/* ------------------------------------------------------------------------- */

/* Covalent part over a short neighbour list (every (j, image) within the
 * largest S of the potential).  Writes per-atom energy (may be NULL) and adds
 * forces into F (n x 3, may be NULL).  Plain double loop over bonds and their
 * k environment; forces by the chain rule through fc, fR, fA, b, zeta_l,
 * cos(theta) and the radial exponential.
 *
 * Charge-dependent coupling (Methods, first paragraph: the covalent-ionic
 * mixed bond nature is expressed by a charge function f_q whose form this
 * paper does not give; the stand-in here): with charges qf != NULL, the
 * attraction of bond (i,j) is scaled by f_q = exp(-kq (q_i - q_j)^2), i.e.
 * the bond energy is 1/2 fc (fR - b fA f_q).  Forces are taken at fixed
 * charges.  cb (may be NULL) receives, for every list entry e of a bond, the
 * charge-free attraction c_e = fc b fA (0 for entries beyond S). */
static SC FN(covalent_q)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L,
                         const double *qf, double kq, double *cb, SC *eat, SC *F)
{
    SC Etot = 0.0;
    (void)n;
    for (int row = 0; row < L->n; row++) {
        const int i = L->rows ? L->rows[row] : row;
        const int ti = types[i];
        const FN(sp_t) *si = &P->sp[ti];
        SC ei = 0.0;
        for (long e = L->off[row]; e < L->off[row + 1]; e++) {
            const int j = L->p[e].j;
            const double r = L->p[e].r;
            FN(pair_t) pj = FN(pair_params)(P, ti, types[j]);
            if (cb) cb[e] = 0.0;
            if (r >= RE(pj.S)) continue;
            const double *dv = L->p[e].d;
            double u[3] = {dv[0] / r, dv[1] / r, dv[2] / r};
            /* environment sums zeta_l (Eq. 2, one per channel) */
            SC z[2] = {0.0, 0.0};
            for (long e2 = L->off[row]; e2 < L->off[row + 1]; e2++) {
                if (e2 == e) continue;
                const int k = L->p[e2].j;
                const double rk = L->p[e2].r;
                FN(pair_t) pk = FN(pair_params)(P, ti, types[k]);
                if (rk >= RE(pk.S)) continue;
                const double *dk = L->p[e2].d;
                double cs = (dv[0] * dk[0] + dv[1] * dk[1] + dv[2] * dk[2]) / (r * rk);
                SC f = FN(fc)(rk, pk.R, pk.S);
                for (int l = 0; l < 2; l++)
                    z[l] += f * FN(wang)(si, l, cs) * FN(eexp)(si->alpha[l], r - rk);
            }
            SC db[2];
            SC b = FN(bond_order)(si, P->p, z, db);
            SC f = FN(fc)(r, pj.R, pj.S), df = FN(dfc)(r, pj.R, pj.S);
            SC fR = pj.A * SEXP(-pj.lam1 * r), fA = pj.B * SEXP(-pj.lam2 * r);
            double fq = 1.0;
            if (qf) {
                const double dq = qf[i] - qf[j];
                fq = exp(-kq * dq * dq);
            }
            if (cb) cb[e] = RE(f * b * fA);
            ei += 0.5 * f * (fR - b * fA * fq);
            if (!F) continue;
            /* pair part: dV/dr at fixed b (and fixed charges) */
            SC dVdr = 0.5 * (df * (fR - b * fA * fq) + f * (-pj.lam1 * fR + b * fq * pj.lam2 * fA));
            for (int a = 0; a < 3; a++) {
                F[3 * i + a] += dVdr * u[a];
                F[3 * j + a] -= dVdr * u[a];
            }
            /* bond-order part: P_l = dV/dzeta_l = -1/2 fc fA f_q db/dzeta_l */
            SC Pl[2] = {-0.5 * f * fA * fq * db[0], -0.5 * f * fA * fq * db[1]};
            for (long e2 = L->off[row]; e2 < L->off[row + 1]; e2++) {
                if (e2 == e) continue;
                const int k = L->p[e2].j;
                const double rk = L->p[e2].r;
                FN(pair_t) pk = FN(pair_params)(P, ti, types[k]);
                if (rk >= RE(pk.S)) continue;
                const double *dk = L->p[e2].d;
                double uk[3] = {dk[0] / rk, dk[1] / rk, dk[2] / rk};
                double cs = u[0] * uk[0] + u[1] * uk[1] + u[2] * uk[2];
                double dcs_dd[3], dcs_dk[3];
                for (int a = 0; a < 3; a++) {
                    dcs_dd[a] = (uk[a] - cs * u[a]) / r;
                    dcs_dk[a] = (u[a] - cs * uk[a]) / rk;
                }
                SC fk = FN(fc)(rk, pk.R, pk.S), dfk = FN(dfc)(rk, pk.R, pk.S);
                for (int l = 0; l < 2; l++) {
                    SC w = FN(wang)(si, l, cs), dw = FN(dwang)(si, l, cs);
                    SC ex = FN(eexp)(si->alpha[l], r - rk), dex = FN(deexp)(si->alpha[l], r - rk);
                    for (int a = 0; a < 3; a++) {
                        /* gradients of this zeta term w.r.t. x_j and x_k */
                        SC gj = fk * dw * ex * dcs_dd[a] + fk * w * dex * u[a];
                        SC gk = dfk * w * ex * uk[a] + fk * dw * ex * dcs_dk[a] - fk * w * dex * uk[a];
                        F[3 * j + a] -= Pl[l] * gj;
                        F[3 * k + a] -= Pl[l] * gk;
                        F[3 * i + a] += Pl[l] * (gj + gk);
                    }
                }
            }
        }
        if (eat) eat[i] = ei;
        Etot += ei;
    }
    return Etot;
}

static SC FN(covalent)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L,
                       SC *eat, SC *F)
{
    return FN(covalent_q)(P, n, types, L, NULL, 0.0, NULL, eat, F);
}

/* ------------------------------------------------------------------------- */
/* charge equilibration                                                      */
/* ------------------------------------------------------------------------- */

/* Off-diagonal Coulomb matrix entries per long-list entry (self images with
 * j == i included; they add to H_ii through the product below). */
static void FN(assemble)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L, SC *Hv)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (long e = L->off[i]; e < L->off[i + 1]; e++)
            Hv[e] = FN(coul)(P, types[i], types[L->p[e].j], L->p[e].r, NULL);
}

/* y = H x with H = diag(J) + Coulomb entries */
static void FN(matvec)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L,
                       const SC *Hv, const SC *x, SC *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) {
        SC s = P->sp[types[i]].J * x[i];
        for (long e = L->off[i]; e < L->off[i + 1]; e++) s += Hv[e] * x[L->p[e].j];
        y[i] = s;
    }
}

/* Projected Jacobi-preconditioned CG for  min chi^T q + 1/2 q^T H q  subject to
 * sum q = Q.  The preconditioned direction z solves the constrained Jacobi
 * system  D z + w 1 = r,  1^T z = 0, i.e. z = D^-1 (r - w 1) with
 * w = (1^T D^-1 r) / (1^T D^-1 1), which keeps every iterate on the constraint.
 * Since 1^T z = 0, r may be shifted by any multiple of 1 without changing the
 * iteration; r is shifted by w every step so that it carries no large
 * constant part (the multiplier mu), which would otherwise swamp r^T z in
 * rounding.  Stops when the RMS of the projected residual is below tol, after
 * confirming it on the recomputed true residual (restarting if it differs);
 * in the complex build the imaginary part, divided by the step h, must also be
 * below tol.  Returns the iteration count, or -1 if maxit was reached. */
static int FN(qeq_solve)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L,
                         const SC *Hv, double Q, double tol, int maxit, double hcs,
                         SC *q, double *res_out, SC *mu_out)
{
    SC *r = calloc(n, sizeof(SC)), *z = calloc(n, sizeof(SC)), *p = calloc(n, sizeof(SC));
    SC *s = calloc(n, sizeof(SC)), *dinv = calloc(n, sizeof(SC));
    /* diagonal of H including self-image entries */
    SC sdinv = 0.0;
    for (int i = 0; i < n; i++) {
        SC d = P->sp[types[i]].J;
        for (long e = L->off[i]; e < L->off[i + 1]; e++)
            if (L->p[e].j == i) d += Hv[e];
        dinv[i] = 1.0 / d;
        sdinv += dinv[i];
    }
    /* start on the constraint */
    SC sq = 0.0;
    for (int i = 0; i < n; i++) sq += q[i];
    for (int i = 0; i < n; i++) q[i] += (Q - sq) / n;
    int it = 0, conv = 0, fresh = 1;
    SC rho = 0.0;
    double res = 0.0;
    for (;;) {
        if (fresh) {       /* (re)start from the true residual */
            FN(matvec)(P, n, types, L, Hv, q, s);
            for (int i = 0; i < n; i++) r[i] = -(s[i] + P->sp[types[i]].chi);
        }
        /* shift r by w; projected residual norm */
        SC srd = 0.0;
        for (int i = 0; i < n; i++) srd += r[i] * dinv[i];
        SC w = srd / sdinv;
        for (int i = 0; i < n; i++) r[i] -= w;
        SC sr = 0.0;
        for (int i = 0; i < n; i++) sr += r[i];
        SC mean = sr / n;
        double nre = 0.0, nim = 0.0;
        for (int i = 0; i < n; i++) {
            SC pr = r[i] - mean;
            nre += RE(pr) * RE(pr);
            nim += IM(pr) * IM(pr);
        }
        res = sqrt(nre / n);
        double resi = (hcs > 0.0) ? sqrt(nim / n) / hcs : 0.0;
        if (res < tol && resi < tol) {
            if (fresh) { conv = 1; break; }
            fresh = 1;       /* confirm on the true residual */
            continue;
        }
        if (it >= maxit) break;
        SC rho_new = 0.0;
        for (int i = 0; i < n; i++) { z[i] = dinv[i] * r[i]; rho_new += r[i] * z[i]; }
        if (fresh) {
            for (int i = 0; i < n; i++) p[i] = z[i];
        } else {
            SC beta = rho_new / rho;
            for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
        fresh = 0;
        rho = rho_new;
        FN(matvec)(P, n, types, L, Hv, p, s);
        SC pAp = 0.0;
        for (int i = 0; i < n; i++) pAp += p[i] * s[i];
        SC alpha = rho / pAp;
        for (int i = 0; i < n; i++) { q[i] += alpha * p[i]; r[i] -= alpha * s[i]; }
        it++;
    }
    /* final exact re-projection onto sum q = Q */
    SC sq2 = 0.0;
    for (int i = 0; i < n; i++) sq2 += q[i];
    for (int i = 0; i < n; i++) q[i] += (Q - sq2) / n;
    /* mu: mean of the gradient chi + H q */
    FN(matvec)(P, n, types, L, Hv, q, s);
    SC mu = 0.0;
    for (int i = 0; i < n; i++) mu += s[i] + P->sp[types[i]].chi;
    if (mu_out) *mu_out = mu / n;
    if (res_out) *res_out = res;
    free(r); free(z); free(p); free(s); free(dinv);
    return conv ? it : -1;
}

/* Coulomb + self energy at given charges; per-atom split into eat (added);
 * Coulomb forces added into F.  Self-image pairs (j == i) give no force. */
static SC FN(charge_terms)(const FN(prm_t) *P, int n, const int *types, const nlist_t *L,
                           const SC *q, SC *eat, SC *F)
{
    SC Etot = 0.0;
    (void)n;
    for (int row = 0; row < L->n; row++) {
        const int i = L->rows ? L->rows[row] : row;
        const FN(sp_t) *s = &P->sp[types[i]];
        SC ei = s->E0 + s->chi * q[i] + 0.5 * s->J * q[i] * q[i];
        for (long e = L->off[row]; e < L->off[row + 1]; e++) {
            const int j = L->p[e].j;
            SC dC;
            SC Cv = FN(coul)(P, types[i], types[j], L->p[e].r, &dC);
            ei += 0.5 * q[i] * q[j] * Cv;
            if (F && j != i) {
                const double r = L->p[e].r;
                for (int a = 0; a < 3; a++) F[3 * i + a] += q[i] * q[j] * dC * L->p[e].d[a] / r;
            }
        }
        if (eat) eat[i] += ei;
        Etot += ei;
    }
    return Etot;
}
