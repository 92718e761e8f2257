/*
 * mobius.h -- C ABI of libmobius.so, the MI355X (gfx950) red/black Moebius
 * domain-wall operator and its conjugate-gradient solver.
 *
 * Operator (Brower, Neff, Orginos, "The Moebius Domain Wall Fermion
 * Algorithm"): the 5d operator D_DW(m) of Sec. 2.1 (block tridiagonal in s,
 * diagonal blocks D+ = b5 D_W + 1, off-diagonal D- P-/P+ with D- = c5 D_W - 1,
 * wall coupling -m D- P+ at (1,Ls) and -m D- P- at (Ls,1)), built on the 4d
 * Wilson operator of Sec. 2
 *     D_W psi(x) = (4 - M5) psi(x)
 *                  - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)]
 * with M5 > 0 the domain-wall height (the paper writes 4 + M5 with M5 = O(-1)).
 * Gamma matrices are in the chiral basis, g5 = diag(1,1,-1,-1), P+ = spins 0,1.
 * Periodic boundaries in all four directions.  An optional chemical potential
 * mu (mobius_params.mu) multiplies the time-like forward hop by e^{+mu} and the
 * backward one by e^{-mu} (Sec. "Baryon current and Chemical Potential").
 *
 * Red/black (Sec. 3): 4d parity (x+y+z+t) mod 2, the same for every s.
 * Parity 0 = even ("red"), parity 1 = odd ("black").  With
 *     I = M+ + M- C5,  M+ = b5 (4 - M5) + 1,  M- = c5 (4 - M5) - 1,
 *     (C5 psi)_s = P+ psi_{s-1} + P- psi_{s+1}  (wrapped neighbours carry -m),
 * the off-diagonal blocks are D_{p,1-p} = -1/2 H_{p,1-p} B with B = b5 + c5 C5
 * (H the Wilson hopping sum on every s-slice), and the preconditioned operator
 * on the odd parity is D_pre = 1 - I^{-1} D_oe I^{-1} D_eo.
 *
 * Conventions of this ABI
 *  - All data pointers are DEVICE pointers on the current HIP device; the
 *    caller owns them.  Nothing here frees caller memory.
 *  - Canonical layouts (complex128, interleaved re/im):
 *        links   [mu=x,y,z,t][t][z][y][x][a][b]        U_mu(x), row a, column b
 *        spinor  [s][t][z][y][x][spin][colour]           s = 0..Ls-1
 *    Multi-RHS calls add a leading [rhs] index.
 *  - Packed half-lattice fields ("packed") are private to the library; their
 *    size in bytes per right-hand side is mobius_field_bytes().  They hold one
 *    parity of a 5d field in the given storage precision.
 *  - Every call enqueues its work on `stream` (a hipStream_t, NULL = default
 *    stream) and returns without synchronising, except mobius_cg_solve,
 *    mobius_batch_solve, mobius_propagator4d, mobius_force and mobius_tune,
 *    which synchronise once at the end to fill their outputs.
 *  - Return codes: MOBIUS_OK (0) on success; MOBIUS_NOT_CONVERGED (1) from
 *    the solver when maxiter is reached (info is still filled); negative codes
 *    on error, with a message in mobius_last_error().  No call aborts or throws.
 *  - in == out aliasing is rejected with MOBIUS_EINVAL.
 */
#ifndef MOBIUS_H
#define MOBIUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOBIUS_OK 0
#define MOBIUS_NOT_CONVERGED 1
#define MOBIUS_EINVAL (-22)
#define MOBIUS_ENOMEM (-12)
#define MOBIUS_EHIP (-100)

/* storage precision of packed fields and links */
typedef enum {
    MOBIUS_F64 = 0, /* FP64 storage and arithmetic */
    MOBIUS_F32 = 1, /* FP32 storage and arithmetic */
    MOBIUS_F16 = 2  /* FP16 storage (spinors scaled by one FP32 max-abs norm per 5d site), FP32 arithmetic */
} mobius_prec;

/* operator selector for mobius_dslash / mobius_dslash_dag */
typedef enum {
    MOBIUS_OP_HOP = 0,   /* off-diagonal block D_{p,1-p} = -1/2 H B: parity 1-p -> p  (Sec. 3) */
    MOBIUS_OP_M5 = 1,    /* diagonal block I on one half field (parity-independent) (Sec. 3)  */
    MOBIUS_OP_SCHUR = 2, /* D_pre = 1 - I^-1 D_oe I^-1 D_eo, odd -> odd (out_parity must be 1)  */
    MOBIUS_OP_FULL = 3,  /* the unpreconditioned D_DW(m) on both halves (Sec. 2.1)            */
    MOBIUS_OP_SCHUR_RIGHT = 4, /* D_R = 1 - D_oe I^-1 D_eo I^-1 = I D_pre I^-1, odd -> odd (Sec. 3,
                                  the diagonal block taken out on the right; out_parity 1) */
    MOBIUS_OP_HOP_LEFT = 5,    /* off-diagonal block of the left form D^ = D-^-1 D_DW D- of
                                  Sec. 2.1: D^_{p,1-p} = -1/2 B H, parity 1-p -> p */
    MOBIUS_OP_SCHUR_LEFT = 6,  /* Schur operator of D^: 1 - I^-1 D^_oe I^-1 D^_eo = B D_pre B^-1,
                                  odd -> odd (out_parity 1) */
    MOBIUS_OP_SCHUR_COMPLEMENT = 7  /* the Schur complement of the even block itself (Sec. 3),
                                  S = I - D_oe I^-1 D_eo = I D_pre, with no diagonal block taken out,
                                  odd -> odd (out_parity 1) */
} mobius_op;

typedef struct {
    int32_t L[4]; /* Lx, Ly, Lz, Lt: each even and >= 2 */
    int32_t Ls;   /* fifth-dimension extent, 2 <= Ls <= 64 */
    double M5;    /* domain-wall height (> 0 in this sign convention) */
    double mf;    /* quark mass m of the wall coupling (0 <= mf <= 1; 1 = Pauli-Villars) */
    double b5;    /* Moebius b5 (Shamir: 1) */
    double c5;    /* Moebius c5 (Shamir: 0) */
    double mu;    /* chemical potential (Sec. "Baryon current and Chemical Potential"): the
                     time-like hops of D_W carry e^{+mu} forward (x -> x + t) and e^{-mu}
                     backward; 0 = none; |mu| <= 10.  The forces differentiate the hops
                     with these factors (gradient with respect to U itself). */
    const double *b5s, *c5s; /* optional HOST arrays of Ls per-slice coefficients b5(s), c5(s),
                     s = 1..Ls, of the general operator of Sec. 2.1 (row s of D_DW holds
                     D+(s) = b5(s) D_W + 1 and D-(s) = c5(s) D_W - 1; e.g. Zolotarev
                     coefficients, Sec. 4.3); read by mobius_create only.  NULL: the
                     constant b5 (c5) above; one NULL and one not: the NULL one constant. */
    int32_t brick[3]; /* site order: bricks of Bx x By x Bz spatial sites, each extended over
                     all t, are the columns the packed traversal (and so every hop's
                     workgroups) walks; each side in 1..L of its direction.  All zero: chosen
                     automatically (the largest brick dividing the lattice whose one-site
                     FP64 slice fits half of one XCD's L2; MOBIUS_BRICK="bx,by,bz" overrides
                     that choice); mobius_tune_brick measures candidates. */
} mobius_params;

typedef struct {
    double tol;            /* target ||eta - D_DW psi|| / ||eta|| (full-system true residual, FP64) */
    int32_t maxiter;       /* cap on CG iterations (all inner iterations counted) */
    int32_t inner_prec;    /* mobius_prec of the CG operator: F64 = plain FP64 CGLS; F32/F16 =
                              low-precision operator with FP64 reductions, reliable updates and
                              outer defect correction */
    double reliable_delta; /* reliable update when ||r|| falls below delta * (max ||r|| since the
                              last update); <= 0 selects the default of the inner precision:
                              0.3 for FP16, 0.1 for FP32 */
    int32_t nrhs;          /* number of right-hand sides in src/sol (>= 1) */
    int32_t check_every;   /* iterations between host convergence checks (<= 0 selects 8 with a
                              lower-precision inner operator, 16 for FP64).  With F32/F16 and
                              check_every <= 16, the FP32 correction to the iterate
                              is updated once per check_every iterations from that many stored
                              search directions (check_every - 1 more inner-precision fields
                              per right-hand side in the context's workspace) */
    double err_tol;        /* > 0: also iterate until err_bound (below) <= err_tol, tightening
                              the Schur target as needed; <= 0: the residual test alone */
    int32_t form;          /* Schur system CGLS iterates on (Sec. 3): 0 = left-preconditioned
                              D_pre psi_o = I^-1 (eta_o - D_oe I^-1 eta_e); 1 = right-preconditioned
                              D_R z = eta_o - D_oe I^-1 eta_e, psi_o = I^-1 z (D_R = I D_pre I^-1);
                              2 = the left form D^ = D-^-1 D_DW D- of Sec. 2.1 (constant b5, c5):
                              (B D_pre B^-1) y = B b', psi_o = B^-1 y, whose hops apply B after
                              the hopping sum and so never gather the s-neighbours of their input;
                              3 = the Schur complement itself, S psi_o = eta_o - D_oe I^-1 eta_e
                              with S = I - D_oe I^-1 D_eo (no diagonal preconditioning).
                              The same solution every way; schur_resid, kappa and err_bound refer
                              to the system iterated on.  mobius_force uses 0. */
} mobius_solve_opts;

typedef struct {
    int32_t iters;        /* CGLS iterations */
    int32_t dirac_apps;   /* hop-kernel applications (4 per CGLS iteration plus source, residual
                             and reconstruction work) */
    int32_t reliable_updates;
    int32_t status;       /* MOBIUS_OK or MOBIUS_NOT_CONVERGED */
    double true_resid;    /* ||eta - D_DW psi|| / ||eta||, recomputed in FP64 after reconstruction */
    double schur_resid;   /* ||b' - D_pre psi_o|| / ||b'|| in FP64 */
    double seconds;       /* wall time of the solve on the stream */
    double algo_bytes;    /* algorithmic HBM bytes of every kernel the solve launched: each field
                             read or written once per launch, links once per hop (no neighbour
                             re-reads, no index tables) */
    double flops;         /* floating-point operations by the same convention (hop: 1416 per
                             5d site, I^-1: 96, vector updates: their multiply-adds) */
    double kappa;         /* estimate of the condition number of D_pre: sqrt(lambda_max /
                             lambda_min) of the Lanczos tridiagonal of D_pre^+ D_pre that the CG
                             coefficients define (extreme Ritz values; 0 if no iteration ran) */
    double err_bound;     /* kappa * schur_resid: bound on ||psi_o - psi_o*|| / ||psi_o*|| of the
                             odd half the CG iterates on (kappa^2 times the residual of the
                             normal equations for mobius_force) */
} mobius_solve_info;

typedef struct mobius_ctx mobius_ctx;

/* Create a context for one lattice and one set of operator parameters.
 * links_c128: device pointer to the canonical links (4*V*9 complex128); the
 * library packs them into context-owned storage (the caller may free its copy
 * after the stream has run).  Returns MOBIUS_EINVAL for odd or < 2 extents,
 * Ls outside [2, 64], a singular Ls-direction block I (M+(s) = 0 for some s,
 * or a vanishing pivot of its cyclic elimination), a non-finite coefficient,
 * or a null pointer. */
int mobius_create(mobius_ctx **ctx, const mobius_params *params, const void *links_c128,
                  void *stream);

/* Release every allocation the context owns.  Synchronises the device. */
int mobius_destroy(mobius_ctx *ctx);

/* Bytes of one packed half-lattice 5d field (one right-hand side) in `prec`. */
int64_t mobius_field_bytes(const mobius_ctx *ctx, int32_t prec);

/* Split a canonical 5d spinor (complex128, nrhs consecutive fields) into its
 * even and odd packed halves in precision `prec` (FP16: per-site norm chosen
 * as the max |component|, round-to-nearest-even). */
int mobius_pack(mobius_ctx *ctx, int32_t prec, const void *canon_c128, void *even, void *odd,
                int32_t nrhs, void *stream);

/* Inverse of mobius_pack: packed halves -> canonical complex128. */
int mobius_unpack(mobius_ctx *ctx, int32_t prec, const void *even, const void *odd,
                  void *canon_c128, int32_t nrhs, void *stream);

/* Apply one red/black block of D_DW to packed fields (Sec. 3):
 *   MOBIUS_OP_HOP   out(parity p) = D_{p,1-p} in(parity 1-p), with
 *                   D_{p,1-p} = -1/2 H_{p,1-p} (b5 + c5 C5): the Wilson hopping
 *                   term on every s-slice after the b5/c5 mixing in s (Sec. 4.1:
 *                   gather s-1, s, s+1, then one Dirac application);
 *   MOBIUS_OP_M5    out = I in (both fields of parity out_parity);
 *   MOBIUS_OP_SCHUR out = D_pre in on the odd parity (out_parity must be 1);
 *   MOBIUS_OP_SCHUR_RIGHT out = D_R in = in - D_oe I^-1 D_eo I^-1 in (odd, out_parity 1);
 *   MOBIUS_OP_FULL  out = D_DW(m) in, the whole 5d operator of Sec. 2.1 (the
 *                   block tridiagonal matrix in s with D+ = b5 D_W + 1 on the
 *                   diagonal), applied on both parities as
 *                   out_p = D_{p,1-p} in_{1-p} + I in_p; out_parity is ignored;
 *   MOBIUS_OP_HOP_LEFT   out(p) = -1/2 B H_{p,1-p} in(1-p), the hop block of the
 *                   left form D^ = D-^-1 D_DW D- = B D_W + 1 - C5 (Sec. 2.1);
 *   MOBIUS_OP_SCHUR_LEFT out = in - I^-1 D^_oe I^-1 D^_eo in (odd, out_parity 1);
 *   MOBIUS_OP_SCHUR_COMPLEMENT out = I in - D_oe I^-1 D_eo in (odd, out_parity 1).
 * The two left-form operators need constant b5, c5 (MOBIUS_EINVAL otherwise:
 * with per-slice coefficients B and I no longer commute) and b5 != 0.
 * in and out are packed fields of precision `prec`, nrhs consecutive fields
 * each; for MOBIUS_OP_FULL each holds 2 nrhs fields: the nrhs even halves, then
 * the nrhs odd halves (the two outputs of mobius_pack placed back to back), and
 * in and out must not overlap. */
int mobius_dslash(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity, const void *in,
                  void *out, int32_t nrhs, void *stream);

/* The same blocks of the adjoint operator D_DW^+:
 *   MOBIUS_OP_HOP   out(p) = (D^+)_{p,1-p} in(1-p) = (D_{1-p,p})^+ in
 *                   = -1/2 B^+ H^+ in, H^+ = H with g_mu -> -g_mu;
 *   MOBIUS_OP_M5    out = I^+ in;
 *   MOBIUS_OP_SCHUR out = D_pre^+ in = in - (D_eo)^+ I^-+ (D_oe)^+ I^-+ in;
 *   MOBIUS_OP_SCHUR_RIGHT out = D_R^+ in = in - I^-+ (D_eo)^+ I^-+ (D_oe)^+ in;
 *   MOBIUS_OP_FULL  out = D_DW(m)^+ in, out_p = (D^+)_{p,1-p} in_{1-p} + I^+ in_p;
 *   MOBIUS_OP_HOP_LEFT   out(p) = (D^_{1-p,p})^+ in = -1/2 H^+ B^+ in;
 *   MOBIUS_OP_SCHUR_LEFT out = in - (D^_eo)^+ I^-+ (D^_oe)^+ I^-+ in;
 *   MOBIUS_OP_SCHUR_COMPLEMENT out = I^+ in - (D_eo)^+ I^-+ (D_oe)^+ in. */
int mobius_dslash_dag(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity,
                      const void *in, void *out, int32_t nrhs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operator blocks of mobius_dslash (dagger = 0) and mobius_dslash_dag
 * (dagger = 1), same arguments and results, with no allocation of any kind.
 * MOBIUS_OP_SCHUR, SCHUR_RIGHT and SCHUR_LEFT keep their two temporary packed
 * fields per right-hand side (HOP_LEFT with dagger = 1 and SCHUR_COMPLEMENT:
 * one) in a fixed
 * workspace of 64 MiB per GPU (a static device array that the library holds
 * from the first mobius_create on that GPU until the process ends); a call
 * needing more (2 * nrhs * mobius_field_bytes(ctx, prec) > 64 MiB) returns
 * MOBIUS_EINVAL.  Every call on one GPU shares that workspace: calls
 * that overlap in time on one GPU (different streams or threads) race and must
 * be serialised by the caller.  Enqueued on stream, like mobius_dslash. */
int mobius_dslash_noalloc(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity,
                          int32_t dagger, const void *in, void *out, int32_t nrhs, void *stream);

/* out = I^{-1} in (dagger = 0) or I^{-+} in (dagger = 1) on a packed half
 * field, by the closed-form elimination of Sec. 3 (I = A P- + A^T P+, each an
 * Ls x Ls cyclic bidiagonal solve per site, spin and colour). */
int mobius_m5inv(mobius_ctx *ctx, int32_t prec, int32_t dagger, const void *in, void *out,
                 int32_t nrhs, void *stream);

/* Solve D_DW(m) psi = eta (Sec. 3 red/black Schur decomposition, CGLS on
 * D_pre, reconstruction of the even half, FP64 true residual).
 * src_c128 / sol_c128: canonical complex128 5d fields, opts->nrhs of them.
 * info: array of opts->nrhs entries.  Returns MOBIUS_OK when every system
 * reached opts->tol, MOBIUS_NOT_CONVERGED otherwise. */
int mobius_cg_solve(mobius_ctx *ctx, const void *src_c128, void *sol_c128,
                    const mobius_solve_opts *opts, mobius_solve_info *info, void *stream);

/* Solve the adjoint system D_DW(m)^+ psi = eta: the red/black decomposition of
 * Sec. 3 applied to D_DW^+ (diagonal blocks I^+, off-diagonal blocks the
 * adjoint hops), CGLS on its left-preconditioned Schur operator
 * 1 - I^-+ (D^+)_oe I^-+ (D^+)_eo (whose adjoint is the right-preconditioned D_R
 * of D_DW), the even half reconstructed, the FP64 true residual
 * ||eta - D_DW^+ psi|| / ||eta||.  Arguments, precisions, reliable updates and
 * return codes as mobius_cg_solve (opts->form is ignored). */
int mobius_cg_solve_dag(mobius_ctx *ctx, const void *src_c128, void *sol_c128,
                        const mobius_solve_opts *opts, mobius_solve_info *info, void *stream);

/* 4d propagator of the overlap operator through the 5d solve (Sec. 2.2):
 *   q = [P^+ D_DW(m)^-1 D_DW(1) P b]_1 = D_ov(m)^-1 b,
 * with the chiral shift P_{ss'} = delta_{ss'} P- + delta_{s',s+1 mod Ls} P+
 * (b enters on the walls: P- b on slice 1, P+ b on slice Ls), D_DW(1) the
 * Pauli-Villars operator (mf = 1, same links and M5, b5, c5) and
 * D_ov(m) = (1+m)/2 + (1-m)/2 g5 eps_Ls(g5 D_Moebius) (App. A).
 * src4_c128 / sol4_c128: canonical complex128 4d fields [t][z][y][x][spin][colour],
 * opts->nrhs of them (device memory, caller-owned).  The 5d solve D_DW(m) psi
 * = D_DW(1) P b runs as mobius_cg_solve with opts; info (opts->nrhs entries)
 * describes it (its true residual is that of the 5d system).  The context
 * keeps two canonical 5d fields and four packed FP64 half fields per
 * right-hand side as temporaries until mobius_destroy.  Returns as
 * mobius_cg_solve. */
int mobius_propagator4d(mobius_ctx *ctx, const void *src4_c128, void *sol4_c128,
                        const mobius_solve_opts *opts, mobius_solve_info *info, void *stream);

/* Overlap to bulk domain-wall reconstruction (Sec. 2.3): given the overlap
 * solution psi = D_ov(m)^-1 b (a 4d field, e.g. from mobius_propagator4d),
 * the 5d field
 *     Psi = P^+ D_DW(m)^-1 D_DW(1) P B,   B = b on slice 1 only,
 * obtained with one Pauli-Villars solve instead of a D_DW(m) solve:
 *     psi~ = psi on slice 1,  y = D_DW(1)^-1 D_DW(m) P psi~,  Omega = P^+ y,
 *     Psi_1 = psi,  Psi_s = -Omega_s  (s = 2..Ls)
 * (P the chiral shift of mobius_propagator4d, (P^+ y)_s = P- y_s + P+ y_{s-1}).
 * The 5d solution of D_DW(m) X = D_DW(1) P B is X = P Psi.
 * psi4_c128: canonical complex128 [t][z][y][x][spin][colour], opts->nrhs of
 * them; Psi5_c128: canonical 5d fields (caller-owned device memory).  The
 * Pauli-Villars solve runs as mobius_cg_solve with opts on a mass-1 view of
 * the context (same links, M5, b5, c5, per-slice coefficients); info (opts->nrhs
 * entries) describes it.  Temporaries (two canonical 5d fields and four packed
 * FP64 half fields per right-hand side, and the view's solver buffers) stay
 * with the context until mobius_destroy.  Returns as mobius_cg_solve. */
int mobius_bulk5d(mobius_ctx *ctx, const void *psi4_c128, void *Psi5_c128,
                  const mobius_solve_opts *opts, mobius_solve_info *info, void *stream);

/* Solve a batch of independent systems on lattices of possibly different
 * sizes (one context each, opts->nrhs right-hand sides per context) in
 * lockstep: every CG step of all systems is one launch (the hop kernels walk
 * the concatenated block lists of all lattices in one persistent launch), so
 * small lattices share the GPU.  src[j], sol[j]: canonical fields of context
 * j; info: n * opts->nrhs entries in context-major order.  The contexts must
 * be distinct.  Returns as mobius_cg_solve. */
int mobius_batch_solve(int32_t n, mobius_ctx *const *ctxs, const void *const *src,
                       void *const *sol, const mobius_solve_opts *opts, mobius_solve_info *info,
                       void *stream);

/* Pseudofermion action of the Schur operator and its derivatives:
 *     S = phi_o^+ (D_pre^+ D_pre)^{-1} phi_o,   X = (D_pre^+ D_pre)^{-1} phi_o,
 * with phi_o the odd-parity part of phi (D_pre as in Sec. 3).  X comes from
 * CG on the normal operator (opts: tol on ||phi_o - D_pre^+ D_pre X|| / ||phi_o||,
 * maxiter, inner_prec with the same FP64 reliable updates as mobius_cg_solve;
 * opts->nrhs must be 0 or 1).  Outputs:
 *   grad_links_c128  canonical links layout (4*V*9 complex128), fully written:
 *                    dS/dRe U + i dS/dIm U for every link entry, treating the
 *                    entries as independent complex numbers (the gradient
 *                    convention of PyTorch for a real function of complex
 *                    inputs; project onto su(3) for a molecular-dynamics force);
 *                    NULL skips the link-derivative pass (S and grad_phi only);
 *   grad_phi_c128    canonical 5d field: dS/dRe phi + i dS/dIm phi = 2 X on
 *                    the odd sites, 0 on the even sites;
 *   action           host pointer receiving S.
 * The link derivative follows dS = -2 Re <D_pre X, dD_pre X>, where only the
 * hopping blocks D_eo, D_oe depend on the links (Sec. 3).  Synchronises once at
 * the end.  Returns MOBIUS_OK, MOBIUS_NOT_CONVERGED (outputs still written
 * from the last iterate) or a negative error code. */
int mobius_force(mobius_ctx *ctx, const void *phi_c128, void *grad_links_c128, void *grad_phi_c128,
                 double *action, const mobius_solve_opts *opts, mobius_solve_info *info,
                 void *stream);

/* 4d Hybrid Monte Carlo action with the pseudofermion on the wall (Sec. 2.4):
 *     S = phi^+ [P^+ D_DW(m)^-1 D_DW(1) D_DW(1)^+ D_DW(m)^-+ P]_{11} phi
 *       = phi^+ (D_ov(m)^+ D_ov(m))^-1 phi,
 * phi a 4d field (P the chiral shift of mobius_propagator4d: phi enters as
 * P- phi on slice 1 and P+ phi on slice Ls), and its link gradient from the
 * two inversions of Sec. 2.4,
 *     chi = D(m)^-+ P phi~ (mobius_cg_solve_dag),  psi = D(m)^-1 D(1) D(1)^+ chi,
 *     S = |D(1)^+ chi|^2,  dS = -2 Re <chi, dD(m) psi> + 2 Re <chi, dD(1) D(1)^+ chi>
 * (dD the change of the hopping part of D_DW, whose wall coupling carries the
 * mass).  phi4_c128: canonical [t][z][y][x][spin][colour] complex128;
 * grad_links_c128: canonical links layout, dS/dRe U + i dS/dIm U per entry as
 * mobius_force (NULL: S only); action: host pointer.  opts as mobius_cg_solve
 * for both solves (nrhs 0 or 1); info receives one record for the pair
 * (iterations and Dirac applications summed, the larger residual, kappa and
 * bound).  Synchronises.  Returns as mobius_cg_solve. */
int mobius_force_wall(mobius_ctx *ctx, const void *phi4_c128, void *grad_links_c128, double *action,
                      const mobius_solve_opts *opts, mobius_solve_info *info, void *stream);

/* Lie-algebra form of a link gradient, for molecular-dynamics updates:
 *   F_mu(x) = TA(U_mu(x) G_mu(x)^+),  TA(M) = (M - M^+)/2 - tr(M - M^+)/6,
 * traceless anti-Hermitian, so that for U -> e^{eps X} U (X in su(3)) the
 * action changes at the rate dS/deps = Re tr(F X).  links_c128, grad_links_c128
 * (G as mobius_force returns it) and lie_c128: canonical [mu][t][z][y][x][a][b]
 * complex128 device arrays of 4 V 3x3 entries; lie_c128 must not alias either
 * input.  Enqueued on stream. */
int mobius_force_lie(mobius_ctx *ctx, const void *links_c128, const void *grad_links_c128,
                     void *lie_c128, void *stream);

/* Launch parameters of the hop kernel chosen by mobius_tune. */
typedef struct {
    int32_t prec;        /* storage precision tuned */
    int32_t prefetch;    /* software-pipelining depth of the direction loop (0, 1, 2) */
    int32_t stage_links; /* links of a workgroup's sites copied to LDS first (0/1) */
    int32_t xcd_remap;   /* workgroups of one XCD cover one contiguous range of sites (0/1) */
    int32_t nt_links;    /* non-temporal link loads (0/1) */
    int32_t mfma;        /* FP16: the colour multiply on the matrix cores (0/1); used with
                            stage_links = 1 when Ls is divisible by 4, ignored otherwise */
    double hop_us;       /* measured time of one hop application D_{p,1-p} (microseconds) */
} mobius_tune_result;

/* Autotune the hop kernel of this context for storage precision `prec`
 * (MOBIUS_F64/F32/F16): every combination of the launch parameters above is
 * timed on `reps` applications of each parity (<= 0 selects 10), the fastest
 * is kept in the context and used by every later call on it (operator blocks,
 * solves, batches, force).  If the environment variable MOBIUS_TUNE_CACHE
 * names a file, an entry for the same lattice, Ls, site order, precision and
 * device is used without timing, and a new measurement is appended to it.
 * The tuner uses context scratch memory only; caller fields are untouched.
 * Synchronises.  out may be NULL. */
int mobius_tune(mobius_ctx *ctx, int32_t prec, int32_t reps, mobius_tune_result *out, void *stream);

/* One candidate site order timed by mobius_tune_brick. */
typedef struct {
    int32_t brick[3]; /* Bx, By, Bz */
    double hop_us;    /* tuned hop time D_{p,1-p} with this site order (microseconds) */
} mobius_brick_trial;

/* Autotune the site order, the tile of sites the hop's workgroups walk, which
 * is fixed for a context at its creation.  Candidates: the automatic brick
 * (first) and the bricks whose sides are half, once or twice its sides and
 * divide the lattice, nearest in volume first, at most 12.  For each, a
 * temporary context is created from p (p->brick ignored) and links_c128, its
 * hop for `prec` is tuned as by mobius_tune (`reps` as there, the same cache
 * file) and its time recorded.  brick_out[3] receives the automatic brick
 * unless a candidate's hop is more than 3 % faster, then the fastest one; us_out
 * (may be NULL) its time; trials (may be NULL, room for max_trials) every
 * candidate in the order timed, *ntrials (may be NULL) how many.  One
 * temporary context (its links in all three precisions) exists at a time.
 * Synchronises.  Create the context to use with p->brick = brick_out. */
int mobius_tune_brick(const mobius_params *p, const void *links_c128, int32_t prec, int32_t reps,
                      mobius_brick_trial *trials, int32_t max_trials, int32_t *ntrials,
                      int32_t *brick_out, double *us_out, void *stream);

/* Set the hop launch parameters of a context for precision t->prec directly
 * (for example those an earlier mobius_tune reported; t->hop_us is ignored).
 * Returns MOBIUS_EINVAL for a value outside the ranges above. */
int mobius_set_tuning(mobius_ctx *ctx, const mobius_tune_result *t);

/* Message of the last error on the calling thread ("" if none). */
const char *mobius_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
