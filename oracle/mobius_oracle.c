/*
 * mobius_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Slow and literal on purpose: each function follows one definition of the
 * paper (cited in its comment), with explicit 4x4 gamma matrices and 3x3 colour
 * products, no spin projection, no blocking and no fusion.  The only
 * parallelism is an OpenMP loop over 4d sites.  See mobius_oracle.h for the
 * layouts and conventions.
 */
#include "mobius_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define NSPIN 4
#define NCOL 3
#define SITE_DOF (NSPIN * NCOL) /* complex numbers per 4d spinor site */

/* ------------------------------------------------------------------------ */
/* lattice geometry                                                          */

static int64_t vol4(const orc_params *p)
{
    return (int64_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
}

static void site_coords(const orc_params *p, int64_t i, int c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int)(i % p->L[mu]);
        i /= p->L[mu];
    }
}

static int64_t site_index(const orc_params *p, const int c[4])
{
    return (((int64_t)c[3] * p->L[2] + c[2]) * p->L[1] + c[1]) * p->L[0] + c[0];
}

/* neighbour x + dir * mu-hat with periodic wrap (dir = +1 or -1) */
static int64_t neighbour(const orc_params *p, int64_t i, int mu, int dir)
{
    int c[4];
    site_coords(p, i, c);
    c[mu] = (c[mu] + dir + p->L[mu]) % p->L[mu];
    return site_index(p, c);
}

static int site_parity(const orc_params *p, int64_t i)
{
    int c[4];
    site_coords(p, i, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* ------------------------------------------------------------------------ */
/* gamma matrices, chiral basis                                              */

static cplx gam[4][NSPIN][NSPIN];

static void init_gammas(void)
{
    static int done = 0;
    if (done) return;
    memset(gam, 0, sizeof(gam));
    /* Pauli matrices */
    cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                gam[k][a][2 + b] = -I * sig[k][a][b]; /* upper-right block -i sigma_k */
                gam[k][2 + a][b] = I * sig[k][a][b];  /* lower-left block  +i sigma_k */
            }
    for (int a = 0; a < 2; ++a) {
        gam[3][a][2 + a] = 1;
        gam[3][2 + a][a] = 1;
    }
    done = 1;
}

/* chirality of spin index: +1 for P+ (spins 0,1), -1 for P- (spins 2,3) */
static int chirality(int spin) { return spin < 2 ? +1 : -1; }

/* ------------------------------------------------------------------------ */
/* 4d building blocks                                                        */

/* v[spin][a] = sum_b M[a][b] w[spin][b]   (M = U or U^+) */
static void colour_mul(const cplx *M, int dagger, const cplx *w, cplx *v)
{
    for (int sp = 0; sp < NSPIN; ++sp)
        for (int a = 0; a < NCOL; ++a) {
            cplx acc = 0;
            for (int b = 0; b < NCOL; ++b) {
                cplx m = dagger ? conj(M[b * NCOL + a]) : M[a * NCOL + b];
                acc += m * w[sp * NCOL + b];
            }
            v[sp * NCOL + a] = acc;
        }
}

/* v = (1 + sign * gamma_mu) w */
static void one_pm_gamma(int mu, double sign, const cplx *w, cplx *v)
{
    for (int sp = 0; sp < NSPIN; ++sp)
        for (int a = 0; a < NCOL; ++a) {
            cplx acc = w[sp * NCOL + a];
            for (int sq = 0; sq < NSPIN; ++sq)
                acc += sign * gam[mu][sp][sq] * w[sq * NCOL + a];
            v[sp * NCOL + a] = acc;
        }
}

/* D_W at one 4d site x.  Wilson operator of Sec. 2 (and App. A):
 *   D_W psi(x) = (4-M5) psi(x) - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu)
 *                                           + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)].
 * Its adjoint, read off as the conjugate transpose of that matrix (gamma_mu
 * Hermitian), swaps the two projectors:
 *   D_W^+ psi(x) = (4-M5) psi(x) - 1/2 sum_mu [(1+g_mu) U_mu(x) psi(x+mu)
 *                                             + (1-g_mu) U_mu(x-mu)^+ psi(x-mu)].
 * A chemical potential multiplies the time-like forward hop of D_W by e^{+mu}
 * and the backward one by e^{-mu}; the adjoint, being the transpose, carries
 * e^{-mu} on its forward and e^{+mu} on its backward time-like hop. */
static void wilson_site(const orc_params *p, const cplx *U, const cplx *in, int64_t x,
                        cplx *out, int dag)
{
    const int64_t V = vol4(p);
    const double sgn = dag ? -1.0 : 1.0;
    cplx v[SITE_DOF], w[SITE_DOF];
    for (int k = 0; k < SITE_DOF; ++k) out[k] = (4.0 - p->M5) * in[x * SITE_DOF + k];
    for (int mu = 0; mu < 4; ++mu) {
        int64_t xf = neighbour(p, x, mu, +1);
        int64_t xb = neighbour(p, x, mu, -1);
        const double ef = mu == 3 ? exp(dag ? -p->mu : p->mu) : 1.0;
        const double eb = mu == 3 ? exp(dag ? p->mu : -p->mu) : 1.0;
        /* forward hop: (1 - sgn g_mu) U_mu(x) psi(x+mu) */
        colour_mul(U + ((int64_t)mu * V + x) * 9, 0, in + xf * SITE_DOF, v);
        one_pm_gamma(mu, -sgn, v, w);
        for (int k = 0; k < SITE_DOF; ++k) out[k] -= 0.5 * ef * w[k];
        /* backward hop: (1 + sgn g_mu) U_mu(x-mu)^+ psi(x-mu) */
        colour_mul(U + ((int64_t)mu * V + xb) * 9, 1, in + xb * SITE_DOF, v);
        one_pm_gamma(mu, +sgn, v, w);
        for (int k = 0; k < SITE_DOF; ++k) out[k] -= 0.5 * eb * w[k];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_wilson(const orc_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    init_gammas();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = vol4(p);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x) wilson_site(p, U, in, x, out + x * SITE_DOF, dag);
}

/* ------------------------------------------------------------------------ */
/* 5d Moebius operator                                                       */

/* Coefficients of row s (0-based) of D_DW: b5(s), c5(s) of the general operator
 * of Sec. 2.1 when per-slice values are given, else the constant ones. */
static double b5_of(const orc_params *p, int s) { return p->b5s ? p->b5s[s] : p->b5; }
static double c5_of(const orc_params *p, int s) { return p->c5s ? p->c5s[s] : p->c5; }

/* chiral projection of a 4d site vector: keep components of chirality `chi` */
static void chiral_part(const cplx *w, int chi, double scale, cplx *acc)
{
    for (int sp = 0; sp < NSPIN; ++sp)
        if (chirality(sp) == chi)
            for (int a = 0; a < NCOL; ++a) acc[sp * NCOL + a] += scale * w[sp * NCOL + a];
}

/* D_DW at 4d site x for every s.  Row s of the block matrix of Sec. 2.1
 * (0-based s here):
 *   out_s = D+ in_s + D- [ P- in_{s+1} + P+ in_{s-1} ],
 * where the wrapped neighbours carry -m (the corners -m D- P+ at (1,Ls) and
 * -m D- P- at (Ls,1)).  D+ = b5 D_W + 1, D- = c5 D_W - 1 act on 4d slices, so
 * D_W is needed on in_s and on the mixed slice w_s at x; they are evaluated
 * with wilson_site on full slices built on the fly.
 *
 * Adjoint: (D^+)_{s,s'} = (D_{s',s})^+.  With y_s = D-(s)^+ in_s (the
 * coefficient of the row the coupling came from):
 *   out_s = D+(s)^+ in_s + P- y_{s-1} + P+ y_{s+1}   (wraps carry -m). */
static void dw_site(const orc_params *p, const cplx *U, const cplx *in, int64_t x, cplx *out,
                    int dag, cplx *slice_buf /* [V][12] scratch */)
{
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
    cplx t1[SITE_DOF], t2[SITE_DOF];
    /* the 9 sites D_W at x reads (x and its 8 neighbours) */
    int64_t nb[9];
    nb[0] = x;
    for (int mu = 0; mu < 4; ++mu) {
        nb[1 + 2 * mu] = neighbour(p, x, mu, +1);
        nb[2 + 2 * mu] = neighbour(p, x, mu, -1);
    }
    for (int s = 0; s < Ls; ++s) {
        cplx *o = out + (int64_t)s * SITE_DOF;
        const cplx *ins = in + (int64_t)s * V * SITE_DOF;
        /* diagonal block D+ (or D+^+) */
        wilson_site(p, U, ins, x, t1, dag);
        for (int k = 0; k < SITE_DOF; ++k) o[k] = b5_of(p, s) * t1[k] + ins[x * SITE_DOF + k];
        if (!dag) {
            /* mixed slice w = P- in_{s+1} + P+ in_{s-1}, needed at the 9 sites */
            int sp1 = (s + 1) % Ls, sm1 = (s - 1 + Ls) % Ls;
            double fp1 = (s == Ls - 1) ? -p->mf : 1.0;
            double fm1 = (s == 0) ? -p->mf : 1.0;
            for (int j = 0; j < 9; ++j) {
                cplx *wb = slice_buf + nb[j] * SITE_DOF;
                memset(wb, 0, sizeof(cplx) * SITE_DOF);
                chiral_part(in + ((int64_t)sp1 * V + nb[j]) * SITE_DOF, -1, fp1, wb);
                chiral_part(in + ((int64_t)sm1 * V + nb[j]) * SITE_DOF, +1, fm1, wb);
            }
            wilson_site(p, U, slice_buf, x, t2, 0);
            for (int k = 0; k < SITE_DOF; ++k)
                o[k] += c5_of(p, s) * t2[k] - slice_buf[x * SITE_DOF + k];
        } else {
            /* y_{s-1} contributes its P- part, y_{s+1} its P+ part */
            int sm1 = (s - 1 + Ls) % Ls, sp1 = (s + 1) % Ls;
            double fm1 = (s == 0) ? -p->mf : 1.0;
            double fp1 = (s == Ls - 1) ? -p->mf : 1.0;
            cplx y[SITE_DOF];
            wilson_site(p, U, in + (int64_t)sm1 * V * SITE_DOF, x, t2, 1);
            for (int k = 0; k < SITE_DOF; ++k)
                y[k] = c5_of(p, sm1) * t2[k] - in[((int64_t)sm1 * V + x) * SITE_DOF + k];
            chiral_part(y, -1, fm1, o);
            wilson_site(p, U, in + (int64_t)sp1 * V * SITE_DOF, x, t2, 1);
            for (int k = 0; k < SITE_DOF; ++k)
                y[k] = c5_of(p, sp1) * t2[k] - in[((int64_t)sp1 * V + x) * SITE_DOF + k];
            chiral_part(y, +1, fp1, o);
        }
    }
}

/* The left form of Sec. 2.1, D^ = D-^{-1} D_DW D- (D- = diag(D-(1), ..., D-(Ls))),
 * which puts the chiral projectors to the left of D-.  Row s (0-based here):
 *   (D^ psi)_s = D+(s) psi_s + P+ D-(s-1) psi_{s-1} + P- D-(s+1) psi_{s+1},
 * the wrapped couplings carrying -m (corners -m P+ D-(Ls) at (1,Ls) and
 * -m P- D-(1) at (Ls,1)).  Adjoint, (D^+)_{s,s'} = (D^_{s',s})^+:
 *   (D^+ psi)_s = D+(s)^+ psi_s + D-(s)^+ (P+ psi_{s+1} + P- psi_{s-1}). */
static void dw_left_site(const orc_params *p, const cplx *U, const cplx *in, int64_t x, cplx *out,
                         int dag, cplx *slice_buf)
{
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
    cplx *W = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);  /* D_W psi_t (or D_W^+) at x */
    for (int t = 0; t < Ls; ++t) wilson_site(p, U, in + (int64_t)t * V * SITE_DOF, x, W + t * SITE_DOF, dag);
    for (int s = 0; s < Ls; ++s) {
        cplx *o = out + (int64_t)s * SITE_DOF;
        const cplx *ps = in + ((int64_t)s * V + x) * SITE_DOF;
        for (int k = 0; k < SITE_DOF; ++k) o[k] = b5_of(p, s) * W[s * SITE_DOF + k] + ps[k];
        const int sm1 = (s - 1 + Ls) % Ls, sp1 = (s + 1) % Ls;
        const double fm1 = (s == 0) ? -p->mf : 1.0, fp1 = (s == Ls - 1) ? -p->mf : 1.0;
        if (!dag) {
            cplx y[SITE_DOF];
            for (int k = 0; k < SITE_DOF; ++k)   /* D-(s-1) psi_{s-1} */
                y[k] = c5_of(p, sm1) * W[sm1 * SITE_DOF + k] - in[((int64_t)sm1 * V + x) * SITE_DOF + k];
            chiral_part(y, +1, fm1, o);
            for (int k = 0; k < SITE_DOF; ++k)   /* D-(s+1) psi_{s+1} */
                y[k] = c5_of(p, sp1) * W[sp1 * SITE_DOF + k] - in[((int64_t)sp1 * V + x) * SITE_DOF + k];
            chiral_part(y, -1, fp1, o);
        } else {
            /* D-(s)^+ applied to the mixed slice w = P+ psi_{s+1} + P- psi_{s-1} */
            int64_t nb[9];
            nb[0] = x;
            for (int mu = 0; mu < 4; ++mu) {
                nb[1 + 2 * mu] = neighbour(p, x, mu, +1);
                nb[2 + 2 * mu] = neighbour(p, x, mu, -1);
            }
            for (int j = 0; j < 9; ++j) {
                cplx *wb = slice_buf + nb[j] * SITE_DOF;
                memset(wb, 0, sizeof(cplx) * SITE_DOF);
                chiral_part(in + ((int64_t)sp1 * V + nb[j]) * SITE_DOF, +1, fp1, wb);
                chiral_part(in + ((int64_t)sm1 * V + nb[j]) * SITE_DOF, -1, fm1, wb);
            }
            cplx t2[SITE_DOF];
            wilson_site(p, U, slice_buf, x, t2, 1);
            for (int k = 0; k < SITE_DOF; ++k)
                o[k] += c5_of(p, s) * t2[k] - slice_buf[x * SITE_DOF + k];
        }
    }
    free(W);
}

void orc_dw_left(const orc_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    init_gammas();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
#pragma omp parallel
    {
        cplx *buf = (cplx *)calloc((size_t)V * SITE_DOF, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);
#pragma omp for schedule(static)
        for (int64_t x = 0; x < V; ++x) {
            dw_left_site(p, U, in, x, tmp, dag, buf);
            for (int s = 0; s < Ls; ++s)
                memcpy(out + ((int64_t)s * V + x) * SITE_DOF, tmp + s * SITE_DOF, sizeof(cplx) * SITE_DOF);
        }
        free(tmp);
        free(buf);
    }
}

/* copy of `in` with the other parity zeroed (in_parity < 0: plain copy) */
static cplx *masked_copy(const orc_params *p, const cplx *in, int in_parity)
{
    const int64_t V = vol4(p);
    const int64_t n = V * p->Ls * SITE_DOF;
    cplx *m = (cplx *)malloc(sizeof(cplx) * n);
    memcpy(m, in, sizeof(cplx) * n);
    if (in_parity >= 0) {
        for (int s = 0; s < p->Ls; ++s)
            for (int64_t x = 0; x < V; ++x)
                if (site_parity(p, x) != in_parity)
                    memset(m + ((int64_t)s * V + x) * SITE_DOF, 0, sizeof(cplx) * SITE_DOF);
    }
    return m;
}

void orc_dw_sites(const orc_params *p, const double *Ud, const double *ind, int in_parity,
                  int64_t nsites, const int64_t *sites, double *outd, int dag)
{
    init_gammas();
    const cplx *U = (const cplx *)Ud;
    cplx *out = (cplx *)outd;
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
    cplx *in = masked_copy(p, (const cplx *)ind, in_parity);
#pragma omp parallel
    {
        cplx *buf = (cplx *)calloc((size_t)V * SITE_DOF, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nsites; ++k) {
            dw_site(p, U, in, sites[k], tmp, dag, buf);
            memcpy(out + k * Ls * SITE_DOF, tmp, sizeof(cplx) * Ls * SITE_DOF);
        }
        free(tmp);
        free(buf);
    }
    free(in);
}

void orc_dw(const orc_params *p, const double *Ud, const double *ind, double *outd, int dag)
{
    init_gammas();
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
#pragma omp parallel
    {
        cplx *buf = (cplx *)calloc((size_t)V * SITE_DOF, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);
#pragma omp for schedule(static)
        for (int64_t x = 0; x < V; ++x) {
            dw_site(p, U, in, x, tmp, dag, buf);
            for (int s = 0; s < Ls; ++s)
                memcpy(out + ((int64_t)s * V + x) * SITE_DOF, tmp + s * SITE_DOF,
                       sizeof(cplx) * SITE_DOF);
        }
        free(tmp);
        free(buf);
    }
}

/* ------------------------------------------------------------------------ */
/* red/black blocks (Sec. 3)                                                 */

static void zero_other_parity(const orc_params *p, cplx *f, int keep_parity)
{
    const int64_t V = vol4(p);
    for (int s = 0; s < p->Ls; ++s)
        for (int64_t x = 0; x < V; ++x)
            if (site_parity(p, x) != keep_parity)
                memset(f + ((int64_t)s * V + x) * SITE_DOF, 0, sizeof(cplx) * SITE_DOF);
}

static int64_t field_len(const orc_params *p) { return vol4(p) * p->Ls * SITE_DOF; }

/* Off-diagonal block: restrict the input to parity 1-q, apply D (or D^+),
 * keep parity q of the result.  This is the definition of D_rb / D_br in the
 * 2x2 block form of Sec. 3. */
void orc_hop(const orc_params *p, const double *U, int out_parity, const double *ind,
             double *outd, int dag)
{
    cplx *m = masked_copy(p, (const cplx *)ind, 1 - out_parity);
    orc_dw(p, U, (const double *)m, outd, dag);
    zero_other_parity(p, (cplx *)outd, out_parity);
    free(m);
}

/* Diagonal blocks I_rr = I_bb: the parity-preserving part of D (or D^+). */
void orc_m5(const orc_params *p, const double *U, const double *ind, double *outd, int dag)
{
    const int64_t n = field_len(p);
    cplx *out = (cplx *)outd;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * n);
    memset(out, 0, sizeof(cplx) * n);
    for (int q = 0; q < 2; ++q) {
        cplx *m = masked_copy(p, (const cplx *)ind, q);
        orc_dw(p, U, (const double *)m, (double *)tmp, dag);
        zero_other_parity(p, tmp, q);
        for (int64_t k = 0; k < n; ++k) out[k] += tmp[k];
        free(m);
    }
    free(tmp);
}

/* Closed-form solves of Sec. 3 with a = M-/M+ and mu = m a (the paper calls
 * them alpha and M; renamed to avoid clashing with the Moebius alpha and M5).
 *
 * A has M+ on the diagonal, M- on the super-diagonal and -m M- at (Ls,1).
 * A psi = b:  psi_Ls = [b_Ls + mu sum_{s=1}^{Ls-1} (-a)^{s-1} b_s] / (M+ (1 - mu (-a)^{Ls-1})),
 *             psi_s  = b_s / M+ - a psi_{s+1},   s = Ls-1, ..., 1.
 * A^T psi = b is the same elimination with rows and columns interchanged
 * (M- on the sub-diagonal, -m M- at (1,Ls)):
 *             psi_1  = [b_1 + mu sum_{s=2}^{Ls} (-a)^{Ls-s} b_s] / (M+ (1 - mu (-a)^{Ls-1})),
 *             psi_s  = b_s / M+ - a psi_{s-1},   s = 2, ..., Ls.
 * b and psi are strided arrays over s (1-based in the formulas, 0-based here). */
static void solve_A(const orc_params *p, double Mp, double Mm, const cplx *b, cplx *psi,
                    int64_t stride, int transpose)
{
    const int Ls = p->Ls;
    const double a = Mm / Mp, mu = p->mf * a;
    const double denom = Mp * (1.0 - mu * pow(-a, Ls - 1));
    if (!transpose) {
        cplx sum = 0;
        for (int s = 1; s <= Ls - 1; ++s) sum += pow(-a, s - 1) * b[(s - 1) * stride];
        psi[(Ls - 1) * stride] = (b[(Ls - 1) * stride] + mu * sum) / denom;
        for (int s = Ls - 1; s >= 1; --s)
            psi[(s - 1) * stride] = b[(s - 1) * stride] / Mp - a * psi[s * stride];
    } else {
        cplx sum = 0;
        for (int s = 2; s <= Ls; ++s) sum += pow(-a, Ls - s) * b[(s - 1) * stride];
        psi[0] = (b[0] + mu * sum) / denom;
        for (int s = 2; s <= Ls; ++s)
            psi[(s - 1) * stride] = b[(s - 1) * stride] / Mp - a * psi[(s - 2) * stride];
    }
}

/* s-dependent coefficients (Sec. 2.1 with the red/black blocks of Sec. 3):
 * the diagonal block of D_DW restricted to one chirality is an Ls x Ls cyclic
 * bidiagonal matrix with d_s = M+(s) = b5(s) (4 - M5) + 1 on the diagonal and
 * M-(s) = c5(s) (4 - M5) - 1 off it:
 *   P-:  "upper" form, M-(s) at (s, s+1), -m M-(Ls) at (Ls, 1);
 *   P+:  "lower" form, M-(s) at (s, s-1), -m M-(1) at (1, Ls);
 * and the adjoint I^+ holds their transposes.  The elimination of Sec. 3
 * carries over with the ratios taken row by row: for the upper form,
 *   psi_1 = S + Q psi_Ls,  S = sum_{s<Ls} g_s b_s / d_s,  g_1 = 1,
 *   g_{s+1} = -g_s e_s / d_s,  Q = g_Ls  (forward elimination),
 *   psi_Ls = (b_Ls - k S) / (d_Ls + k Q)  (k the corner),
 *   psi_s = (b_s - e_s psi_{s+1}) / d_s,  s = Ls-1, ..., 1  (back substitution);
 * the lower form is its mirror image in s.  e[s] holds the off-diagonal
 * element of row s (unused where the row has none). */
static void solve_upper(int Ls, const double *d, const double *e, double k, const cplx *b, cplx *psi,
                        int64_t st)
{
    cplx S = 0;
    double g = 1.0;
    for (int s = 0; s < Ls - 1; ++s) {
        S += g * b[s * st] / d[s];
        g *= -e[s] / d[s];
    }
    psi[(Ls - 1) * st] = (b[(Ls - 1) * st] - k * S) / (d[Ls - 1] + k * g);
    for (int s = Ls - 2; s >= 0; --s) psi[s * st] = (b[s * st] - e[s] * psi[(s + 1) * st]) / d[s];
}

static void solve_lower(int Ls, const double *d, const double *e, double k, const cplx *b, cplx *psi,
                        int64_t st)
{
    cplx S = 0;
    double g = 1.0;
    for (int s = Ls - 1; s > 0; --s) {
        S += g * b[s * st] / d[s];
        g *= -e[s] / d[s];
    }
    psi[0] = (b[0] - k * S) / (d[0] + k * g);
    for (int s = 1; s < Ls; ++s) psi[s * st] = (b[s * st] - e[s] * psi[(s - 1) * st]) / d[s];
}

static void m5inv_general(const orc_params *p, const cplx *in, cplx *out, int dag)
{
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
    double *Mp = (double *)malloc(sizeof(double) * Ls), *Mm = (double *)malloc(sizeof(double) * Ls);
    double *em = (double *)malloc(sizeof(double) * Ls), *ep = (double *)malloc(sizeof(double) * Ls);
    for (int s = 0; s < Ls; ++s) {
        Mp[s] = b5_of(p, s) * (4.0 - p->M5) + 1.0;
        Mm[s] = c5_of(p, s) * (4.0 - p->M5) - 1.0;
    }
    /* off-diagonal element of each row and the corner, per chirality */
    double km, kp;
    if (!dag) {  /* I:   P- upper (row s: M-(s)),   P+ lower (row s: M-(s)) */
        for (int s = 0; s < Ls; ++s) em[s] = ep[s] = Mm[s];
        km = -p->mf * Mm[Ls - 1];
        kp = -p->mf * Mm[0];
    } else {     /* I^+: P- lower (row s: M-(s-1)), P+ upper (row s: M-(s+1)) */
        for (int s = 0; s < Ls; ++s) {
            em[s] = s > 0 ? Mm[s - 1] : 0.0;
            ep[s] = s < Ls - 1 ? Mm[s + 1] : 0.0;
        }
        km = -p->mf * Mm[Ls - 1];
        kp = -p->mf * Mm[0];
    }
    const int64_t stride = V * SITE_DOF;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x)
        for (int sp = 0; sp < NSPIN; ++sp)
            for (int a = 0; a < NCOL; ++a) {
                const int64_t off = x * SITE_DOF + sp * NCOL + a;
                const int minus = chirality(sp) < 0;
                const int upper = minus != dag;
                if (upper)
                    solve_upper(Ls, Mp, minus ? em : ep, minus ? km : kp, in + off, out + off, stride);
                else
                    solve_lower(Ls, Mp, minus ? em : ep, minus ? km : kp, in + off, out + off, stride);
            }
    free(Mp);
    free(Mm);
    free(em);
    free(ep);
}

/* I^{-1} = A^{-1} P- + A^{-T} P+ (Sec. 3), with M+ = b5 (4 - M5) + 1 and
 * M- = c5 (4 - M5) - 1.  The adjoint I^{-+} = A^{-T} P- + A^{-1} P+ since A is
 * real.  Applied independently at every 4d site, spin and colour. */
void orc_m5inv(const orc_params *p, const double *ind, double *outd, int dag)
{
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    if (p->b5s || p->c5s) {
        m5inv_general(p, in, out, dag);
        return;
    }
    const int64_t V = vol4(p);
    const double Mp = p->b5 * (4.0 - p->M5) + 1.0;
    const double Mm = p->c5 * (4.0 - p->M5) - 1.0;
    const int64_t stride = V * SITE_DOF;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < V; ++x)
        for (int sp = 0; sp < NSPIN; ++sp)
            for (int a = 0; a < NCOL; ++a) {
                int64_t off = x * SITE_DOF + sp * NCOL + a;
                int minus = chirality(sp) < 0;
                int transpose = dag ? minus : !minus;
                solve_A(p, Mp, Mm, in + off, out + off, stride, transpose);
            }
}

/* D_pre = 1 - I^{-1} D_oe I^{-1} D_eo on the odd parity (Sec. 3, left
 * preconditioned Schur complement with red = even, black = odd).
 * D_pre^+ = 1 - (D_eo)^+ I^{-+} (D_oe)^+ I^{-+}, where (D_eo)^+ is the
 * odd <- even block of D^+ and (D_oe)^+ its even <- odd block. */
void orc_schur(const orc_params *p, const double *U, const double *ind, double *outd, int dag)
{
    const int64_t n = field_len(p);
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t2 = (cplx *)malloc(sizeof(cplx) * n);
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    if (!dag) {
        orc_hop(p, U, 0, ind, (double *)t1, 0);           /* D_eo x      (even) */
        orc_m5inv(p, (double *)t1, (double *)t2, 0);      /* I^-1        (even) */
        orc_hop(p, U, 1, (double *)t2, (double *)t1, 0);  /* D_oe        (odd)  */
        orc_m5inv(p, (double *)t1, (double *)t2, 0);      /* I^-1        (odd)  */
    } else {
        cplx *xo = masked_copy(p, in, 1);
        orc_m5inv(p, (double *)xo, (double *)t1, 1);      /* I^-+        (odd)  */
        orc_hop(p, U, 0, (double *)t1, (double *)t2, 1);  /* (D_oe)^+    (even) */
        orc_m5inv(p, (double *)t2, (double *)t1, 1);      /* I^-+        (even) */
        orc_hop(p, U, 1, (double *)t1, (double *)t2, 1);  /* (D_eo)^+    (odd)  */
        free(xo);
    }
    for (int64_t k = 0; k < n; ++k) out[k] = in[k] - t2[k];
    zero_other_parity(p, out, 1);
    free(t1);
    free(t2);
}

/* ------------------------------------------------------------------------ */
/* CGLS                                                                      */

static double norm2(const cplx *v, int64_t n)
{
    double s = 0;
    for (int64_t k = 0; k < n; ++k) s += creal(v[k]) * creal(v[k]) + cimag(v[k]) * cimag(v[k]);
    return s;
}

/* Right-preconditioned Schur operator on the odd parity (the same Schur
 * decomposition of Sec. 3 with the diagonal block taken out on the right):
 *   D_R = 1 - D_oe I^{-1} D_eo I^{-1} = I D_pre I^{-1},
 *   D_R^+ = 1 - I^{-+} (D_eo)^+ I^{-+} (D_oe)^+.
 * D_R^+ is also the left-preconditioned Schur operator of the adjoint matrix
 * D_DW^+ (whose blocks are I^+ and the adjoint hops). */
static void schur_right(const orc_params *p, const double *U, const cplx *in, cplx *out, int dag)
{
    const int64_t n = field_len(p);
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t2 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *xo = masked_copy(p, in, 1);
    if (!dag) {
        orc_m5inv(p, (double *)xo, (double *)t1, 0);      /* I^-1        (odd)  */
        orc_hop(p, U, 0, (double *)t1, (double *)t2, 0);  /* D_eo        (even) */
        orc_m5inv(p, (double *)t2, (double *)t1, 0);      /* I^-1        (even) */
        orc_hop(p, U, 1, (double *)t1, (double *)t2, 0);  /* D_oe        (odd)  */
    } else {
        orc_hop(p, U, 0, (double *)xo, (double *)t1, 1);  /* (D_oe)^+    (even) */
        orc_m5inv(p, (double *)t1, (double *)t2, 1);      /* I^-+        (even) */
        orc_hop(p, U, 1, (double *)t2, (double *)t1, 1);  /* (D_eo)^+    (odd)  */
        orc_m5inv(p, (double *)t1, (double *)t2, 1);      /* I^-+        (odd)  */
    }
    for (int64_t k = 0; k < n; ++k) out[k] = xo[k] - t2[k];
    zero_other_parity(p, out, 1);
    free(t1);
    free(t2);
    free(xo);
}

void orc_schur_right(const orc_params *p, const double *U, const double *in, double *out, int dag)
{
    schur_right(p, U, (const cplx *)in, (cplx *)out, dag);
}

/* operators CGLS iterates on: 0 = D_pre (left), 1 = D_DW, 2 = D_R (right),
 * 3 = the left Schur operator of D_DW^+, i.e. D_R^+ (with dag: D_R) */
static void apply_op(const orc_params *p, const double *U, int which, const cplx *in, cplx *out,
                     int dag)
{
    if (which == 0)
        orc_schur(p, U, (const double *)in, (double *)out, dag);
    else if (which == 1)
        orc_dw(p, U, (const double *)in, (double *)out, dag);
    else if (which == 2)
        schur_right(p, U, in, out, dag);
    else
        schur_right(p, U, in, out, !dag);
}

/* Conjugate gradient on the normal equations A^+ A x = A^+ b (CGLS form):
 *   x = 0, r = b, s = A^+ r, p = s, gamma = |s|^2;
 *   repeat: q = A p; alpha = gamma/|q|^2; x += alpha p; r -= alpha q;
 *           s = A^+ r; gamma' = |s|^2; p = s + (gamma'/gamma) p; gamma = gamma'
 *   until |r| <= tol |b|.  The paper only says "conjugate gradient" (Sec. 4.1). */
void orc_cgls(const orc_params *p, const double *U, int which, const double *bd, double *xd,
              double tol, int32_t maxiter, orc_info *info)
{
    const int64_t n = field_len(p);
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = (cplx *)malloc(sizeof(cplx) * n);
    cplx *s = (cplx *)malloc(sizeof(cplx) * n);
    cplx *pv = (cplx *)malloc(sizeof(cplx) * n);
    cplx *q = (cplx *)malloc(sizeof(cplx) * n);
    memset(x, 0, sizeof(cplx) * n);
    memcpy(r, b, sizeof(cplx) * n);
    apply_op(p, U, which, r, s, 1);
    memcpy(pv, s, sizeof(cplx) * n);
    double gamma = norm2(s, n);
    const double bnorm = sqrt(norm2(b, n));
    double rnorm = bnorm;
    int it = 0, conv = 0;
    if (bnorm == 0.0) conv = 1;
    while (!conv && it < maxiter) {
        apply_op(p, U, which, pv, q, 0);
        const double alpha = gamma / norm2(q, n);
        for (int64_t k = 0; k < n; ++k) {
            x[k] += alpha * pv[k];
            r[k] -= alpha * q[k];
        }
        ++it;
        rnorm = sqrt(norm2(r, n));
        if (rnorm <= tol * bnorm) {
            conv = 1;
            break;
        }
        apply_op(p, U, which, r, s, 1);
        const double gnew = norm2(s, n);
        const double beta = gnew / gamma;
        for (int64_t k = 0; k < n; ++k) pv[k] = s[k] + beta * pv[k];
        gamma = gnew;
    }
    if (info) {
        info->iters = it;
        info->converged = conv;
        info->rel_resid = bnorm > 0 ? rnorm / bnorm : 0.0;
        info->true_resid = -1.0;
    }
    free(r);
    free(s);
    free(pv);
    free(q);
}

/* Red/black solve of D_DW psi = eta through the Schur (LDU) factorisation of
 * Sec. 3:  b' = I^{-1}(eta_o - D_oe I^{-1} eta_e);  D_pre psi_o = b';
 *          psi_e = I^{-1}(eta_e - D_eo psi_o). */
void orc_solve(const orc_params *p, const double *U, const double *etad, double *psid,
               double tol, int32_t maxiter, orc_info *info)
{
    const int64_t n = field_len(p);
    const cplx *eta = (const cplx *)etad;
    cplx *psi = (cplx *)psid;
    cplx *ee = masked_copy(p, eta, 0);
    cplx *eo = masked_copy(p, eta, 1);
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t2 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *xo = (cplx *)malloc(sizeof(cplx) * n);

    orc_m5inv(p, (double *)ee, (double *)t1, 0);           /* I^-1 eta_e        */
    orc_hop(p, U, 1, (double *)t1, (double *)t2, 0);       /* D_oe I^-1 eta_e   */
    for (int64_t k = 0; k < n; ++k) t2[k] = eo[k] - t2[k];
    orc_m5inv(p, (double *)t2, (double *)t1, 0);           /* b'                */
    zero_other_parity(p, t1, 1);

    orc_cgls(p, U, 0, (double *)t1, (double *)xo, tol, maxiter, info);

    orc_hop(p, U, 0, (double *)xo, (double *)t2, 0);       /* D_eo psi_o        */
    for (int64_t k = 0; k < n; ++k) t2[k] = ee[k] - t2[k];
    orc_m5inv(p, (double *)t2, (double *)t1, 0);           /* psi_e             */
    zero_other_parity(p, t1, 0);
    for (int64_t k = 0; k < n; ++k) psi[k] = t1[k] + xo[k];

    /* true residual of the full system */
    orc_dw(p, U, (double *)psi, (double *)t2, 0);
    for (int64_t k = 0; k < n; ++k) t2[k] = eta[k] - t2[k];
    if (info) {
        double en = sqrt(norm2(eta, n));
        info->true_resid = en > 0 ? sqrt(norm2(t2, n)) / en : 0.0;
    }
    free(ee);
    free(eo);
    free(t1);
    free(t2);
    free(xo);
}

/* Red/black solves in the other forms of the same Schur decomposition:
 *  form 1 (right): z = I psi_o,  D_R z = eta_o - D_oe I^{-1} eta_e,
 *                  psi_o = I^{-1} z,  psi_e = I^{-1}(eta_e - D_eo psi_o);
 *  form 2 (adjoint system D_DW^+ psi = eta): the decomposition of D_DW^+, whose
 *                  diagonal blocks are I^+ and off-diagonal blocks the adjoint
 *                  hops ((D^+)_{oe} = (D_eo)^+ maps even to odd):
 *                  b'_o = I^{-+}(eta_o - (D^+)_{oe} I^{-+} eta_e),
 *                  (1 - I^{-+} (D^+)_{oe} I^{-+} (D^+)_{eo}) psi_o = b'_o,
 *                  psi_e = I^{-+}(eta_e - (D^+)_{eo} psi_o).
 * info->true_resid is that of the system solved (D_DW or D_DW^+). */
void orc_solve_form(const orc_params *p, const double *U, const double *etad, double *psid,
                    double tol, int32_t maxiter, int form, orc_info *info)
{
    if (form == 0) {
        orc_solve(p, U, etad, psid, tol, maxiter, info);
        return;
    }
    const int64_t n = field_len(p);
    const cplx *eta = (const cplx *)etad;
    cplx *psi = (cplx *)psid;
    const int dg = form == 2;
    cplx *ee = masked_copy(p, eta, 0);
    cplx *eo = masked_copy(p, eta, 1);
    cplx *t1 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t2 = (cplx *)malloc(sizeof(cplx) * n);
    cplx *xo = (cplx *)malloc(sizeof(cplx) * n);

    orc_m5inv(p, (double *)ee, (double *)t1, dg);          /* I^-1 eta_e (I^-+)       */
    orc_hop(p, U, 1, (double *)t1, (double *)t2, dg);      /* odd <- even block       */
    for (int64_t k = 0; k < n; ++k) t2[k] = eo[k] - t2[k];
    zero_other_parity(p, t2, 1);
    if (form == 1) {
        orc_cgls(p, U, 2, (double *)t2, (double *)t1, tol, maxiter, info);  /* z     */
        orc_m5inv(p, (double *)t1, (double *)xo, 0);                        /* psi_o */
    } else {
        orc_m5inv(p, (double *)t2, (double *)t1, 1);                        /* b'_o  */
        zero_other_parity(p, t1, 1);
        orc_cgls(p, U, 3, (double *)t1, (double *)xo, tol, maxiter, info);
    }
    zero_other_parity(p, xo, 1);
    orc_hop(p, U, 0, (double *)xo, (double *)t2, dg);      /* even <- odd block       */
    for (int64_t k = 0; k < n; ++k) t2[k] = ee[k] - t2[k];
    orc_m5inv(p, (double *)t2, (double *)t1, dg);          /* psi_e                   */
    zero_other_parity(p, t1, 0);
    for (int64_t k = 0; k < n; ++k) psi[k] = t1[k] + xo[k];
    orc_dw(p, U, (double *)psi, (double *)t2, dg);
    for (int64_t k = 0; k < n; ++k) t2[k] = eta[k] - t2[k];
    if (info) {
        double en = sqrt(norm2(eta, n));
        info->true_resid = en > 0 ? sqrt(norm2(t2, n)) / en : 0.0;
    }
    free(ee);
    free(eo);
    free(t1);
    free(t2);
    free(xo);
}

/* ------------------------------------------------------------------------ */
/* pseudofermion action and its link derivative                              */

/* Plain conjugate gradient (Hestenes-Stiefel) on the Hermitian positive
 * operator A = D_pre^+ D_pre of the odd parity:
 *   x = 0, r = phi, p = r;
 *   repeat: q = A p; alpha = |r|^2 / <p, q>; x += alpha p; r -= alpha q;
 *           beta = |r'|^2 / |r|^2; p = r' + beta p
 *   until |r| <= tol |phi|.  <p, q> = |D_pre p|^2 is evaluated as such. */
void orc_cgne(const orc_params *p, const double *U, const double *phid, double *xd, double tol,
              int32_t maxiter, orc_info *info)
{
    const int64_t n = field_len(p);
    cplx *phi = masked_copy(p, (const cplx *)phid, 1);
    cplx *x = (cplx *)xd;
    cplx *r = (cplx *)malloc(sizeof(cplx) * n);
    cplx *pv = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t = (cplx *)malloc(sizeof(cplx) * n);
    cplx *q = (cplx *)malloc(sizeof(cplx) * n);
    memset(x, 0, sizeof(cplx) * n);
    memcpy(r, phi, sizeof(cplx) * n);
    memcpy(pv, phi, sizeof(cplx) * n);
    const double pnorm = sqrt(norm2(phi, n));
    double rr = norm2(r, n);
    int it = 0, conv = pnorm == 0.0;
    while (!conv && it < maxiter) {
        orc_schur(p, U, (const double *)pv, (double *)t, 0);
        orc_schur(p, U, (const double *)t, (double *)q, 1);
        const double alpha = rr / norm2(t, n);
        for (int64_t k = 0; k < n; ++k) {
            x[k] += alpha * pv[k];
            r[k] -= alpha * q[k];
        }
        ++it;
        const double rr_new = norm2(r, n);
        if (sqrt(rr_new) <= tol * pnorm) {
            rr = rr_new;
            conv = 1;
            break;
        }
        const double beta = rr_new / rr;
        for (int64_t k = 0; k < n; ++k) pv[k] = r[k] + beta * pv[k];
        rr = rr_new;
    }
    if (info) {
        info->iters = it;
        info->converged = conv;
        info->rel_resid = pnorm > 0 ? sqrt(rr) / pnorm : 0.0;
        info->true_resid = -1.0;
    }
    free(phi);
    free(r);
    free(pv);
    free(t);
    free(q);
}

/* 2 Re <a, D[E] b> restricted to the 4d sites of the list: D[E] is D_DW
 * evaluated with the link field E on an input b that vanishes on the parity
 * of those sites, i.e. the hopping term alone (the site-diagonal parts of D+,
 * D- and of the s coupling see only b at the site itself, which is zero). */
static double hop_overlap(const orc_params *p, const cplx *E, const cplx *a, const cplx *b,
                          const int64_t *sites, int nsites, cplx *tmp, cplx *buf)
{
    const int64_t V = vol4(p);
    double acc = 0.0;
    for (int j = 0; j < nsites; ++j) {
        dw_site(p, E, b, sites[j], tmp, 0, buf);
        for (int s = 0; s < p->Ls; ++s)
            for (int k = 0; k < SITE_DOF; ++k)
                acc += 2.0 * creal(conj(a[((int64_t)s * V + sites[j]) * SITE_DOF + k]) *
                                   tmp[s * SITE_DOF + k]);
    }
    return acc;
}

/* S = phi^+ (D_pre^+ D_pre)^{-1} phi for phi on the odd parity, and its
 * derivative with respect to the gauge links.
 *
 * With X = (D_pre^+ D_pre)^{-1} phi and Y = D_pre X, a change of the links
 * changes S by dS = -2 Re <Y, dD_pre X>.  I does not depend on the links, so
 *   dD_pre = -I^-1 dD_oe I^-1 D_eo - I^-1 D_oe I^-1 dD_eo
 * and  dS = 2 Re <Yt, dD_oe Z> + 2 Re <W, dD_eo X>  with
 *   Yt = I^-+ Y (odd),  Z = I^-1 D_eo X (even),  W = I^-+ (D_oe)^+ Yt (even).
 * The off-diagonal blocks are real-linear in the links (they hold the whole
 * link dependence of D_DW, Sec. 3), so the change of D_oe along a direction
 * E is the block itself built on the link field E.  For link l = mu*V + y the
 * directional derivative along E = e_ab (one complex entry set to 1) and
 * along E = i e_ab gives
 *   grad[l][a][b] = dS/dRe U + i dS/dIm U
 * (PyTorch's convention for the gradient of a real function of complex
 * entries).  Only the sites y and y + mu see link l.
 *
 * links: nlinks indices mu*V + y, or NULL for all 4 V links in canonical
 * order (grad then has the canonical link layout).  X (full-size, zero on the
 * even parity) receives the CG solution.  Returns S. */
double orc_force(const orc_params *p, const double *U, const double *phid, double *xd,
                 int64_t nlinks, const int64_t *links, double *gradd, double tol,
                 int32_t maxiter, orc_info *info)
{
    init_gammas();
    const int64_t n = field_len(p);
    const int64_t V = vol4(p);
    cplx *X = (cplx *)xd;
    cplx *grad = (cplx *)gradd;
    orc_cgne(p, U, phid, xd, tol, maxiter, info);

    cplx *Y = (cplx *)malloc(sizeof(cplx) * n);
    cplx *Yt = (cplx *)malloc(sizeof(cplx) * n);
    cplx *Z = (cplx *)malloc(sizeof(cplx) * n);
    cplx *W = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t = (cplx *)malloc(sizeof(cplx) * n);
    orc_schur(p, U, xd, (double *)Y, 0);                 /* Y  = D_pre X            */
    orc_m5inv(p, (double *)Y, (double *)Yt, 1);          /* Yt = I^-+ Y     (odd)   */
    orc_hop(p, U, 0, xd, (double *)t, 0);                /* D_eo X          (even)  */
    orc_m5inv(p, (double *)t, (double *)Z, 0);           /* Z  = I^-1 D_eo X        */
    orc_hop(p, U, 0, (double *)Yt, (double *)t, 1);      /* (D_oe)^+ Yt     (even)  */
    orc_m5inv(p, (double *)t, (double *)W, 1);           /* W  = I^-+ (D_oe)^+ Yt   */

    const cplx *phi = (const cplx *)phid;
    double S = 0.0;
    for (int64_t k = 0; k < n; ++k) S += creal(conj(phi[k]) * X[k]);
    /* (phi restricted to the odd parity: X vanishes on the even one) */

    const int64_t nl = links ? nlinks : 4 * V;
#pragma omp parallel
    {
        cplx *E = (cplx *)calloc((size_t)4 * V * 9, sizeof(cplx));
        cplx *buf = (cplx *)calloc((size_t)V * SITE_DOF, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * p->Ls * SITE_DOF);
#pragma omp for schedule(dynamic, 4)
        for (int64_t l = 0; l < nl; ++l) {
            const int64_t lid = links ? links[l] : l;
            const int mu = (int)(lid / V);
            const int64_t y = lid % V;
            const int64_t sites[2] = {y, neighbour(p, y, mu, +1)};
            for (int e = 0; e < 9; ++e) {
                double d[2];
                for (int part = 0; part < 2; ++part) {
                    E[lid * 9 + e] = part ? I : 1.0;
                    double acc = 0.0;
                    for (int j = 0; j < 2; ++j) {
                        if (site_parity(p, sites[j]) == 1)  /* odd row: dD_oe on Z */
                            acc += hop_overlap(p, E, Yt, Z, &sites[j], 1, tmp, buf);
                        else                                /* even row: dD_eo on X */
                            acc += hop_overlap(p, E, W, X, &sites[j], 1, tmp, buf);
                    }
                    d[part] = acc;
                    E[lid * 9 + e] = 0.0;
                }
                grad[l * 9 + e] = d[0] + I * d[1];
            }
        }
        free(E);
        free(buf);
        free(tmp);
    }
    free(Y);
    free(Yt);
    free(Z);
    free(W);
    free(t);
    return S;
}

/* ------------------------------------------------------------------------ */
/* 4d-HMC action with the pseudofermion on the wall (Sec. 2.4)               */

/* 2 Re <a, H[E] b> summed over the listed 4d sites, H[E] the hopping part of
 * D_DW built on the link field E (D_DW[E] - D_DW[0]: the link-free diagonal
 * parts cancel). */
static double hopping_overlap(const orc_params *p, const cplx *E, const cplx *Z, const cplx *a,
                              const cplx *b, const int64_t *sites, int nsites, cplx *tmp,
                              cplx *tmp0, cplx *buf)
{
    const int64_t V = vol4(p);
    double acc = 0.0;
    for (int j = 0; j < nsites; ++j) {
        dw_site(p, E, b, sites[j], tmp, 0, buf);
        dw_site(p, Z, b, sites[j], tmp0, 0, buf);
        for (int s = 0; s < p->Ls; ++s)
            for (int k = 0; k < SITE_DOF; ++k)
                acc += 2.0 * creal(conj(a[((int64_t)s * V + sites[j]) * SITE_DOF + k]) *
                                   (tmp[s * SITE_DOF + k] - tmp0[s * SITE_DOF + k]));
    }
    return acc;
}

/* S = phi^+ [P^+ D(m)^-1 D(1) D(1)^+ D(m)^-+ P]_{11} phi for a 4d pseudofermion
 * phi on the wall (slice 1 of the propagator matrix: P phi~, phi~ = phi on s = 1),
 * which equals phi^+ (D_ov^+ D_ov)^-1 phi.  With
 *   chi = D(m)^-+ P phi~,   psi = D(m)^-1 D(1) D(1)^+ chi,
 * S = |D(1)^+ chi|^2 and a change of the links changes it by
 *   dS = -2 Re <chi, dD(m) psi> + 2 Re <chi, dD(1) D(1)^+ chi>
 * (the two inversions of Sec. 2.4; dD the change of the hopping part, which
 * depends on the mass through the wall coupling of B).  The gradient per link
 * entry follows orc_force: directional derivatives along e_ab and i e_ab. */
double orc_force_wall(const orc_params *p, const double *Ud, const double *phid, int64_t nlinks,
                      const int64_t *links, double *gradd, double tol, int32_t maxiter,
                      orc_info *info)
{
    init_gammas();
    const cplx *phi = (const cplx *)phid;
    cplx *grad = (cplx *)gradd;
    const int64_t n = field_len(p);
    const int64_t V = vol4(p);
    const int Ls = p->Ls;
    orc_params pv = *p;
    pv.mf = 1.0;
    cplx *w = (cplx *)calloc((size_t)n, sizeof(cplx));
    cplx *chi = (cplx *)malloc(sizeof(cplx) * n);
    cplx *d1c = (cplx *)malloc(sizeof(cplx) * n);
    cplx *t = (cplx *)malloc(sizeof(cplx) * n);
    cplx *psi = (cplx *)malloc(sizeof(cplx) * n);
    /* P phi~: P- phi on slice 1, P+ phi on slice Ls */
    for (int64_t x = 0; x < V; ++x)
        for (int sp = 0; sp < NSPIN; ++sp)
            for (int a = 0; a < NCOL; ++a) {
                const int64_t k = x * SITE_DOF + sp * NCOL + a;
                const int s = chirality(sp) < 0 ? 0 : Ls - 1;
                w[(int64_t)s * V * SITE_DOF + k] = phi[k];
            }
    orc_info i1, i2;
    orc_solve_form(p, Ud, (double *)w, (double *)chi, tol, maxiter, 2, &i1);  /* D(m)^+ chi = P phi~ */
    orc_dw(&pv, Ud, (double *)chi, (double *)d1c, 1);                         /* D(1)^+ chi          */
    orc_dw(&pv, Ud, (double *)d1c, (double *)t, 0);                           /* D(1) D(1)^+ chi     */
    orc_solve(p, Ud, (double *)t, (double *)psi, tol, maxiter, &i2);          /* psi                 */
    const double S = norm2(d1c, n);
    if (info) {
        info->iters = i1.iters + i2.iters;
        info->converged = i1.converged && i2.converged;
        info->rel_resid = fmax(i1.rel_resid, i2.rel_resid);
        info->true_resid = fmax(i1.true_resid, i2.true_resid);
    }
    const int64_t nl = links ? nlinks : 4 * V;
#pragma omp parallel
    {
        cplx *E = (cplx *)calloc((size_t)4 * V * 9, sizeof(cplx));
        cplx *Z = (cplx *)calloc((size_t)4 * V * 9, sizeof(cplx));
        cplx *buf = (cplx *)calloc((size_t)V * SITE_DOF, sizeof(cplx));
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);
        cplx *tmp0 = (cplx *)malloc(sizeof(cplx) * Ls * SITE_DOF);
#pragma omp for schedule(dynamic, 4)
        for (int64_t l = 0; l < nl; ++l) {
            const int64_t lid = links ? links[l] : l;
            const int mu = (int)(lid / V);
            const int64_t y = lid % V;
            const int64_t at[2] = {y, neighbour(p, y, mu, +1)};  /* the rows link l enters */
            for (int e = 0; e < 9; ++e) {
                double d[2];
                for (int part = 0; part < 2; ++part) {
                    E[lid * 9 + e] = part ? I : 1.0;
                    d[part] = -hopping_overlap(p, E, Z, chi, psi, at, 2, tmp, tmp0, buf) +
                              hopping_overlap(&pv, E, Z, chi, d1c, at, 2, tmp, tmp0, buf);
                    E[lid * 9 + e] = 0.0;
                }
                grad[l * 9 + e] = d[0] + I * d[1];
            }
        }
        free(E);
        free(Z);
        free(buf);
        free(tmp);
        free(tmp0);
    }
    free(w);
    free(chi);
    free(d1c);
    free(t);
    free(psi);
    return S;
}
