/*
 * mobius_oracle.h -- plain FP64 CPU oracle for the Moebius domain-wall operator
 * (Brower, Neff, Orginos, "The Moebius Domain Wall Fermion Algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source, header, table or helper
 * with the HIP path.
 *
 * Every field is in the natural ("canonical") layout, complex128:
 *   gauge links  U[mu][t][z][y][x][a][b]        mu = 0..3 for x,y,z,t
 *   4d spinor    psi[t][z][y][x][spin][colour]
 *   5d spinor    psi[s][t][z][y][x][spin][colour]   s = 0..Ls-1 (paper's s = 1..Ls)
 * Parity of a 4d site = (x+y+z+t) mod 2; parity 0 is "red" (even), parity 1
 * "black" (odd).  Half-lattice fields are full-size arrays that are zero on
 * the other parity.
 *
 * Conventions (the readings of the paper that the oracle fixes):
 *  - Wilson operator (Sec. 2, eq. for D^Wilson; App. A):
 *      D_W psi(x) = (4 - M5) psi(x)
 *                   - 1/2 sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *    with M5 > 0 the domain-wall height (the paper writes 4+M5 with M5 = O(-1)
 *    but quotes M5 = 1.8, 1.5; the kernel bound (8-M5)/(10-M5) of Sec. 2 fixes
 *    the sign).  Periodic in all four directions.
 *  - Chiral gamma basis: g_k = [[0,-i s_k],[i s_k,0]], g_4 = [[0,1],[1,0]],
 *    g5 = g1 g2 g3 g4 = diag(1,1,-1,-1); P+ = spins {0,1}, P- = spins {2,3}.
 *  - D_DW(m): the Ls x Ls tridiagonal block matrix of Sec. 2.1 (eq. MoebiusOp):
 *    row s holds D+(s) = b5(s) D_W + 1 on the diagonal, D-(s) P- at (s,s+1),
 *    D-(s) P+ at (s,s-1), -m D-(1) P+ at (1,Ls) and -m D-(Ls) P- at (Ls,1),
 *    D-(s) = c5(s) D_W - 1 (constant b5, c5 unless per-slice values are given).
 */
#ifndef MOBIUS_ORACLE_H
#define MOBIUS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t L[4];   /* Lx, Ly, Lz, Lt (all even, >= 2) */
    int32_t Ls;     /* fifth-dimension extent (>= 2) */
    double  M5;     /* domain-wall height; D_W diagonal is 4 - M5 */
    double  mf;     /* quark mass m of the wall coupling */
    double  b5, c5; /* Moebius coefficients, constant in s */
    double  mu;     /* chemical potential: time-like hops carry e^{+mu} (forward) and
                       e^{-mu} (backward) (Sec. "Baryon current and Chemical Potential") */
    const double *b5s, *c5s; /* optional per-slice coefficients b5(s), c5(s), s = 1..Ls
                       (Ls values each; the general operator of Sec. 2.1 with
                       D+(s) = b5(s) D_W + 1, D-(s) = c5(s) D_W - 1); NULL: the
                       constant b5, c5 above */
} orc_params;

typedef struct {
    int32_t iters;       /* CG iterations taken */
    int32_t converged;   /* 1 if the stopping test was met */
    double  rel_resid;   /* final ||r||/||b|| of the system CG iterated on */
    double  true_resid;  /* ||eta - D_DW psi|| / ||eta|| (full solves only) */
} orc_info;

/* number of OpenMP threads the oracle runs with, and a way to change it */
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* 4d Wilson operator D_W (dag = 0) or its adjoint D_W^+ (dag = 1). */
void orc_wilson(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* 5d Moebius domain-wall operator D_DW(m) (dag = 0) or D_DW(m)^+ (dag = 1). */
void orc_dw(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* D_DW (or D_DW^+) evaluated only at the listed 4d sites (all s, all spin and
 * colour).  `sites` holds canonical 4d indices; out is [nsites][Ls][4][3].
 * If in_parity is 0 or 1, `in` is treated as zero on the other parity. */
void orc_dw_sites(const orc_params *p, const double *U, const double *in, int in_parity,
                  int64_t nsites, const int64_t *sites, double *out, int dag);

/* Red/black blocks of Sec. 3.  Off-diagonal block of D_DW (dag = 0) or of
 * D_DW^+ (dag = 1) that maps parity 1-out_parity to out_parity. */
void orc_hop(const orc_params *p, const double *U, int out_parity, const double *in,
             double *out, int dag);

/* Diagonal block I (= I_rr = I_bb), applied on both parities. */
void orc_m5(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* I^{-1} (dag = 0) or I^{-+} (dag = 1) by the closed-form elimination of Sec. 3
 * (constant coefficients) or its O(Ls) generalisation to s-dependent ones. */
void orc_m5inv(const orc_params *p, const double *in, double *out, int dag);

/* Schur complement D_pre = 1 - I^{-1} D_oe I^{-1} D_eo on the odd parity
 * (dag = 1: its adjoint).  in/out are odd-parity fields. */
void orc_schur(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* CGLS on D_pre (which = 0) or on the unpreconditioned D_DW (which = 1):
 * solves A x = b in the least-squares sense, stopping when ||b - A x|| <= tol ||b||. */
void orc_cgls(const orc_params *p, const double *U, int which, const double *b, double *x,
              double tol, int32_t maxiter, orc_info *info);

/* Full red/black solve of D_DW psi = eta (Sec. 3): source preparation,
 * CGLS on D_pre to Schur tolerance tol, reconstruction of the even half,
 * and the true residual. */
void orc_solve(const orc_params *p, const double *U, const double *eta, double *psi,
               double tol, int32_t maxiter, orc_info *info);

/* Conjugate gradient on D_pre^+ D_pre X = phi (phi on the odd parity; the
 * even parity of phi is ignored).  info->rel_resid is |phi - A X| / |phi| as
 * iterated. */
void orc_cgne(const orc_params *p, const double *U, const double *phi, double *X, double tol,
              int32_t maxiter, orc_info *info);

/* S = phi^+ (D_pre^+ D_pre)^{-1} phi and dS/dU for the listed links
 * (mu * V + canonical 4d index; links = NULL: all links, canonical order).
 * grad[l][a][b] = dS/dRe U_l[a][b] + i dS/dIm U_l[a][b] (complex128).
 * X receives (D_pre^+ D_pre)^{-1} phi.  Returns S. */
double orc_force(const orc_params *p, const double *U, const double *phi, double *X,
                 int64_t nlinks, const int64_t *links, double *grad, double tol,
                 int32_t maxiter, orc_info *info);

/* The left form D^ = D-^{-1} D_DW D- of Sec. 2.1 (chiral projectors to the left
 * of D-): row s holds D+(s) psi_s + P+ D-(s-1) psi_{s-1} + P- D-(s+1) psi_{s+1}
 * (wrapped couplings -m); dag = 1 applies its adjoint. */
void orc_dw_left(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* Right-preconditioned Schur operator D_R = 1 - D_oe I^{-1} D_eo I^{-1} (dag = 1:
 * its adjoint) on odd-parity fields. */
void orc_schur_right(const orc_params *p, const double *U, const double *in, double *out, int dag);

/* Red/black solve in another form of the Schur decomposition: form 0 = left
 * (orc_solve), 1 = right-preconditioned (D_R z = ..., psi_o = I^{-1} z),
 * 2 = the adjoint system D_DW^+ psi = eta (left form of the decomposition of
 * D_DW^+).  info->true_resid is that of the system solved. */
void orc_solve_form(const orc_params *p, const double *U, const double *eta, double *psi,
                    double tol, int32_t maxiter, int form, orc_info *info);

/* 4d-HMC action of Sec. 2.4 with the pseudofermion on the wall:
 * S = phi^+ [P^+ D(m)^-1 D(1) D(1)^+ D(m)^-+ P]_{11} phi (phi a 4d field
 * [t][z][y][x][4][3]) and dS/dU for the listed links (as orc_force), from the
 * two inversions chi = D(m)^-+ P phi~ and psi = D(m)^-1 D(1) D(1)^+ chi. */
double orc_force_wall(const orc_params *p, const double *U, const double *phi, int64_t nlinks,
                      const int64_t *links, double *grad, double tol, int32_t maxiter,
                      orc_info *info);

#ifdef __cplusplus
}
#endif
#endif
