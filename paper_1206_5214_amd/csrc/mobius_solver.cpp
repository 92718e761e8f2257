// mobius_solver.cpp -- red/black CGLS for one or many systems at once.
//
// A "system" is one right-hand side on one lattice; a "group" is one lattice
// (context) with its nrhs systems.  All systems of a solve iterate in
// lockstep: every CG step is a handful of launches that cover every system
// (the hop kernels stage each block's links in LDS once and reuse them for
// all right-hand sides of the group; with several groups the hop is one
// persistent launch over the concatenated block lists of all lattices).
// Every system has its own CG scalars in device memory and an active flag
// honoured by every kernel, so converged systems stop costing bandwidth.
//
// Algorithm per system (Sec. 3 and Sec. 4.1 of the paper; CGLS on the
// normal equations of the Schur operator):
//   b' = I^-1 (eta_o - D_oe I^-1 eta_e)
//   CGLS on D_pre x = b' with the operator and Krylov vectors in precision lo,
//     FP64 reductions, x accumulated in a correction x_lo (FP32 for FP16);
//   reliable update (lo != FP64): when |r| < delta * |r| at the last update,
//     x_hi += x_lo and r = b' - D_pre x_hi in FP64; if that did not at least
//     halve the true residual, the next direction restarts (beta = 0:
//     defect correction);
//   when |r| reaches the Schur target: psi_e = I^-1 (eta_e - D_eo x_hi) and
//   the FP64 true residual |eta - D_DW psi| / |eta|; below tol the system is
//   done, otherwise its Schur target is tightened and it continues.
// Iterations run in chunks of check_every captured in a hipGraph (the host
// looks at the residuals only between chunks).
#include "mobius_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace mobius {
namespace {

#define CK(expr)                                                                                  \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return set_error(MOBIUS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

int env_int(const char *name, int dflt)
{
    const char *e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

// fields of a group (each holds nrhs consecutive packed fields)
enum Field { F_ETA_E, F_ETA_O, F_B, F_XH, F_RH, F_T64, F_U64, F_Q64, F_PE, F_PO,  // FP64
             F_X,                                                          // correction
             F_R, F_P, F_Q, F_S, F_T, F_U,                                 // precision lo
             NFIELDS, F_NONE = -1 };

// CG iterations whose coefficients are kept for the condition-number estimate
constexpr int64_t HIST_MAX = 8192;

struct Group {
    mobius_ctx *ctx;
    int nrhs, sys0;
    const char *src;
    char *sol;
    int64_t fb[NFIELDS];      // bytes of one field of each kind
    char *f[NFIELDS];         // (f[F_P]: the ring slot of the current iteration)
    char *pring;              // slot 0 of the ring of directions
    int64_t hop_blocks, blas_blocks;
};

// extra per-system doubles
enum Extra { X_BNORM2 = 0, X_RES_E = 2, X_RES_O = 3, X_HR = 4, X_ETA_E2 = 5, X_ETA_O2 = 6,
             X_ACTION = 7, X_MINUS1 = 8, NEXTRA = 16 };

struct HopPattern {
    int prec, dag, epi, out_parity;
    Field in, out, x, y;
    bool norm;
};

// hop call patterns: D0A/D0B = D_pre p (norm), D1B/D1C = D_pre^+ r (norm),
// H0A/H0B = D_pre x_hi in FP64; normal equations: D1Q = D_pre^+ q (no norm),
// N64B/N64C = D_pre^+ of an FP64 field
enum HopPid { HP_D0A, HP_D0B, HP_D1B, HP_D1C, HP_H0A, HP_H0B, HP_D1Q, HP_N64B, HP_N64C, NHOP };
enum VecPid { VP_CONV_RH_R, VP_ACC, VP_RES, VP_HOPRED, VP_BLASRED, VP_NORM_B,
              VP_NORM_EE, VP_NORM_EO, VP_CONV_B_RH, VP_XR_N, VP_PUPD_N, VP_RES_N, VP_DOT_B_XH,
              VP_TWO_XH, VP_PUPD_X, VP_XFLUSH, VP_RUPD, VP_NORM_Q, VP_NORM_S, VP_NORM_T64, VP_NORM_Q64,
              VP_PUPD_R, VP_XRING, VP_PUPD_RN, VP_R_N, NVEC };

// Outputs of a force evaluation (normal-equations mode, one system).
struct ForceOut {
    void *grad_links;  // canonical complex128 [4][V][3][3]
    void *grad_phi;    // canonical complex128 5d field
    double action;
};

struct Batch {
    std::vector<Group> groups;
    int nsys = 0;
    int lo = MOBIUS_F64, px = MOBIUS_F64;
    // Deferred x update: with ring > 1 the directions of one chunk of `ring`
    // iterations go to consecutive slots of a ring (iteration q of a chunk
    // writes p to slot q, reading the previous one from slot q - 1, or from
    // slot ring - 1 at q = 0), and x += sum_q alpha_q p_q runs once at the
    // chunk's end: the FP32 x is read and written once per chunk instead of
    // once per iteration.  ring = 1: x += alpha p_old in every iteration.
    int ring = 1;
    hipStream_t st = nullptr;
    int64_t pstride = 0, max_n5 = 0, max_site_blocks = 0;
    // device state (in the first context's buffers)
    double *part = nullptr;
    CgScalars *sc = nullptr;
    double *hist = nullptr;         // [nsys][HIST_MAX][2] CG coefficients (kappa estimate)
    double *extra = nullptr;
    int32_t *active = nullptr, *restart = nullptr;
    HopParams *hop_tab = nullptr;   // [NHOP][ngroups]
    // several lattices with a ring of directions: the D0A and D0B descriptors
    // of each slot (p read from that slot), [ring][2][ngroups]
    HopParams *hop_ring_tab = nullptr;
    std::vector<HopParams> h_hop_ring;
    int cur_slot = 0;               // ring slot of the iteration being issued
    VecSys *vec_tab = nullptr;      // [NVEC][nsys]
    int64_t *prefix = nullptr;      // [NHOP][ngroups + 1]
    size_t hop_lds[NHOP] = {};
    int hop_pf[NHOP] = {};          // loop variant of each batched launch
    int batch_grid = 0;
    HopPattern hp[NHOP];
    // host mirrors
    std::vector<int32_t> h_active, h_restart;
    std::vector<HopParams> h_hop;
    std::vector<VecSys> h_vec;
    std::vector<int64_t> h_prefix;
    // normal: CG on D_pre^+ D_pre x = b (b = the odd half of the source)
    // instead of CGLS for D_DW psi = eta
    bool normal = false;
    // form of the Schur system CGLS iterates on (FORM_LEFT: D_pre; FORM_RIGHT:
    // D_R = I D_pre I^-1 on z = I psi_o; FORM_LHAT: B D_pre B^-1 on y = B psi_o;
    // FORM_ADJ: the left form of the adjoint matrix, for D_DW^+ psi = eta)
    int form = FORM_LEFT;
    bool adj() const { return form == FORM_ADJ; }
    // field holding psi_o (the right form iterates on z = I psi_o, the left
    // form of D^ on y = B psi_o)
    Field psi_o() const { return form == FORM_RIGHT || form == FORM_LHAT ? F_PO : F_XH; }
    // what the r update solves on the new residual: I^-+ r for the left
    // form's adjoint hops, I^-1 r for the adjoint system's, B^+ I^-+ r for the
    // left form of D^, nothing for the right form
    int rupd_mode() const
    {
        return form == FORM_LEFT ? 0 : form == FORM_ADJ ? 1 : form == FORM_LHAT ? 3 : 2;  // 2: right, plain
    }
    // accounting (count_only: account a graph replay without launching)
    bool count_only = false;
    // |out|^2 partial sums fused into the epilogue of the hops that produce q
    // and s (false: the hop without them, then a separate norm pass)
    bool fused_norm = true;

    int dirac = 0;
    double abytes = 0, aflops = 0;

    int ngroups() const { return (int)groups.size(); }
    int nactive() const
    {
        int n = 0;
        for (int j = 0; j < nsys; ++j) n += h_active[j] != 0;
        return n;
    }
    double sum_fb(int prec, bool active_only) const
    {
        double b = 0;
        for (const Group &g : groups)
            for (int r = 0; r < g.nrhs; ++r)
                if (!active_only || h_active[g.sys0 + r]) b += (double)field_bytes(g.ctx->g, prec);
        return b;
    }
    double sum_n5(bool active_only) const
    {
        double n = 0;
        for (const Group &g : groups)
            for (int r = 0; r < g.nrhs; ++r)
                if (!active_only || h_active[g.sys0 + r]) n += (double)g.ctx->g.N5;
        return n;
    }
    double sum_links(int prec) const
    {
        double b = 0;
        for (const Group &g : groups) b += 72.0 * g.ctx->g.Vh * link_elem_bytes(prec);
        return b;
    }

    int setup(mobius_ctx *const *ctxs, int n, const void *const *src, void *const *sol, int nrhs,
              int prec);
    HopArgs hop_args_for(const Group &g, const HopPattern &p) const;
    hipError_t hop(int pid);
    hipError_t launch_pattern(const HopPattern &p, int pid);
    int norm_red() const { return fused_norm ? VP_HOPRED : VP_BLASRED; }
    hipError_t hop_group(const Group &g, int prec, int dag, int epi, int out_parity, Field in,
                         Field out, Field x, Field y, bool norm);
    hipError_t vec(int pid, int kind, int prec, int prec2, bool all = false);
    hipError_t ring_vec(int pid, int kind, int a0, int a1);
    hipError_t reduce(int pid, double *out, int64_t stride, bool all = false);
    hipError_t m5inv_dag_all(int prec, Field in, Field out, bool only_active = false)
    {
        return m5inv_all(prec, 1, in, out, only_active);
    }
    hipError_t m5inv_all(int prec, int dag, Field in, Field out, bool only_active = false,
                         bool bmix = false);
    hipError_t next_u(bool only_active);   // the solve of r the next step's A^+ starts from
    hipError_t psi_odd();                  // psi_o from the iterate (right form: I^-1 z)
    hipError_t body(int q, int k);       // iteration q of a chunk of k CG iterations
    hipError_t rupd();                   // r -= alpha q (|r|^2), u = I^-+ r
    hipError_t body_normal(int q, int k);  // the same on the normal equations
    hipError_t reliable_update();        // x_hi += x, r = b - D x_hi (FP64), r_lo = r
    hipError_t finalize_group(const Group &g);
    int fetch(std::vector<double> &out, int which);
    int kappa(std::vector<double> &out);  // Lanczos estimate of cond(D_pre) per system
    void acct_hop(int prec, int epi, double fields, double n5);
};

int Batch::setup(mobius_ctx *const *ctxs, int n, const void *const *src, void *const *sol,
                 int nrhs, int prec)
{
    lo = prec;
    px = prec == MOBIUS_F16 ? MOBIUS_F32 : prec;
    groups.resize(n);
    nsys = 0;
    for (int j = 0; j < n; ++j) {
        Group &g = groups[j];
        g.ctx = ctxs[j];
        g.nrhs = nrhs;
        g.sys0 = nsys;
        nsys += nrhs;
        g.src = static_cast<const char *>(src[j]);
        g.sol = static_cast<char *>(sol[j]);
        const Geometry &G = g.ctx->g;
        for (int k = 0; k < NFIELDS; ++k)
            g.fb[k] = field_bytes(G, k <= F_PO ? MOBIUS_F64 : k == F_X ? px : lo);
        // p: `ring` slots of nrhs fields each
        auto slots = [&](int k) { return k == F_P ? (int64_t)ring : 1; };
        int64_t need = 4096;
        for (int k = 0; k < NFIELDS; ++k) need += g.fb[k] * nrhs * slots(k);
        CK(g.ctx->work.ensure(need));
        char *w = static_cast<char *>(g.ctx->work.p);
        for (int k = 0; k < NFIELDS; ++k) {
            g.f[k] = w;
            w += g.fb[k] * nrhs * slots(k);
        }
        g.pring = g.f[F_P];
        g.hop_blocks = site_kernel_blocks(G);
        max_site_blocks = std::max(max_site_blocks, g.hop_blocks);
        g.blas_blocks = blas_blocks(G);
        pstride = std::max(pstride, std::max(g.hop_blocks, g.blas_blocks));
        max_n5 = std::max(max_n5, G.N5);
    }
    // |out|^2 partial sums fused into the hop epilogue for every system (the
    // FP16 corruption once seen with several right-hand sides came from the
    // store-data hazard that the buffer-store guard now covers);
    // MOBIUS_SPLIT_NORM=1 takes them in a separate pass instead
    fused_norm = env_int("MOBIUS_SPLIT_NORM", 0) == 0;
    // hop call patterns of the iteration and of the reliable update
    // t = B I^-1 D_eo p, so that the second hop reads its input already mixed in s
    hp[HP_D0A] = {lo, 0, EPI_M5INV | EPI_BMIX, 0, F_P, F_T, F_NONE, F_NONE, false};
    hp[HP_D0B] = {lo, 0, EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB | EPI_NORM, 1, F_T, F_Q, F_P, F_NONE, true};
    hp[HP_D1B] = {lo, 1, EPI_M5INV, 0, F_U, F_T, F_NONE, F_NONE, false};
    hp[HP_D1C] = {lo, 1, EPI_POSTSUB | EPI_NORM, 1, F_T, F_S, F_R, F_NONE, true};
    hp[HP_H0A] = {MOBIUS_F64, 0, EPI_M5INV, 0, F_XH, F_T64, F_NONE, F_NONE, false};
    hp[HP_H0B] = {MOBIUS_F64, 0, EPI_M5INV | EPI_POSTSUB, 1, F_T64, F_Q64, F_XH, F_NONE, false};
    if (form == FORM_RIGHT) {
        // A = D_R = 1 - D_oe I^-1 D_eo I^-1: q = p - D_oe t, t = B I^-1 D_eo v, v = I^-1 p (in u);
        // A^+ = 1 - I^-+ D_eo^+ I^-+ D_oe^+: s = r - I^-+ D_eo^+ t, t = I^-+ D_oe^+ r
        hp[HP_D0A] = {lo, 0, EPI_M5INV | EPI_BMIX, 0, F_U, F_T, F_NONE, F_NONE, false};
        hp[HP_D0B] = {lo, 0, EPI_PREMIXED | EPI_POSTSUB | EPI_NORM, 1, F_T, F_Q, F_P, F_NONE, true};
        hp[HP_D1B] = {lo, 1, EPI_M5INV, 0, F_R, F_T, F_NONE, F_NONE, false};
        hp[HP_D1C] = {lo, 1, EPI_M5INV | EPI_POSTSUB | EPI_NORM, 1, F_T, F_S, F_R, F_NONE, true};
        hp[HP_H0A] = {MOBIUS_F64, 0, EPI_M5INV, 0, F_U64, F_T64, F_NONE, F_NONE, false};
        hp[HP_H0B] = {MOBIUS_F64, 0, EPI_POSTSUB, 1, F_T64, F_Q64, F_XH, F_NONE, false};
    } else if (form == FORM_ADJ) {
        // D_DW^+: A = 1 - I^-+ (D^+)_oe I^-+ (D^+)_eo (adjoint hops, I^-+ epilogues),
        // A^+ = D_R of D_DW, applied to r through u = I^-1 r
        hp[HP_D0A] = {lo, 1, EPI_M5INV, 0, F_P, F_T, F_NONE, F_NONE, false};
        hp[HP_D0B] = {lo, 1, EPI_M5INV | EPI_POSTSUB | EPI_NORM, 1, F_T, F_Q, F_P, F_NONE, true};
        hp[HP_D1B] = {lo, 0, EPI_M5INV | EPI_BMIX, 0, F_U, F_T, F_NONE, F_NONE, false};
        hp[HP_D1C] = {lo, 0, EPI_PREMIXED | EPI_POSTSUB | EPI_NORM, 1, F_T, F_S, F_R, F_NONE, true};
        hp[HP_H0A] = {MOBIUS_F64, 1, EPI_M5INV, 0, F_XH, F_T64, F_NONE, F_NONE, false};
        hp[HP_H0B] = {MOBIUS_F64, 1, EPI_M5INV | EPI_POSTSUB, 1, F_T64, F_Q64, F_XH, F_NONE, false};
    } else if (form == FORM_PLAIN) {
        // A = S = I - D_oe I^-1 D_eo: q = I p - D_oe t, t = B I^-1 D_eo p;
        // A^+ = I^+ - D_eo^+ I^-+ D_oe^+: s = I^+ r - D_eo^+ t, t = I^-+ D_oe^+ r
        hp[HP_D0A] = {lo, 0, EPI_M5INV | EPI_BMIX, 0, F_P, F_T, F_NONE, F_NONE, false};
        hp[HP_D0B] = {lo, 0, EPI_PREMIXED | EPI_M5SUB | EPI_NORM, 1, F_T, F_Q, F_NONE, F_P, true};
        hp[HP_D1B] = {lo, 1, EPI_M5INV, 0, F_R, F_T, F_NONE, F_NONE, false};
        hp[HP_D1C] = {lo, 1, EPI_M5SUB | EPI_NORM, 1, F_T, F_S, F_NONE, F_R, true};
        hp[HP_H0A] = {MOBIUS_F64, 0, EPI_M5INV | EPI_BMIX, 0, F_XH, F_T64, F_NONE, F_NONE, false};
        hp[HP_H0B] = {MOBIUS_F64, 0, EPI_PREMIXED | EPI_M5SUB, 1, F_T64, F_Q64, F_NONE, F_XH, false};
    } else if (form == FORM_LHAT) {
        // A = 1 - I^-1 D^_oe I^-1 D^_eo with D^ = -1/2 B H: q = p - I^-1 B (-1/2 H t),
        // t = I^-1 B (-1/2 H p); A^+ = 1 - (D^_eo)^+ I^-+ (D^_oe)^+ I^-+:
        // s = r - (-1/2 H^+ t), t = B^+ I^-+ (-1/2 H^+ u), u = B^+ I^-+ r
        constexpr int FW = EPI_PREMIXED | EPI_M5INV | EPI_BMIX;
        hp[HP_D0A] = {lo, 0, FW, 0, F_P, F_T, F_NONE, F_NONE, false};
        hp[HP_D0B] = {lo, 0, FW | EPI_POSTSUB | EPI_NORM, 1, F_T, F_Q, F_P, F_NONE, true};
        hp[HP_D1B] = {lo, 1, EPI_NOBOUT | EPI_M5INV | EPI_BMIX, 0, F_U, F_T, F_NONE, F_NONE, false};
        hp[HP_D1C] = {lo, 1, EPI_NOBOUT | EPI_POSTSUB | EPI_NORM, 1, F_T, F_S, F_R, F_NONE, true};
        hp[HP_H0A] = {MOBIUS_F64, 0, FW, 0, F_XH, F_T64, F_NONE, F_NONE, false};
        hp[HP_H0B] = {MOBIUS_F64, 0, FW | EPI_POSTSUB, 1, F_T64, F_Q64, F_XH, F_NONE, false};
    }
    hp[HP_D1Q] = {lo, 1, EPI_POSTSUB, 1, F_T, F_S, F_Q, F_NONE, false};
    hp[HP_N64B] = {MOBIUS_F64, 1, EPI_M5INV, 0, F_U64, F_T64, F_NONE, F_NONE, false};
    hp[HP_N64C] = {MOBIUS_F64, 1, EPI_POSTSUB, 1, F_T64, F_PE, F_Q64, F_NONE, false};

    // device state in the first context
    mobius_ctx *c0 = groups[0].ctx;
    CK(c0->partials.ensure((int64_t)nsys * pstride * (int64_t)sizeof(double)));
    part = static_cast<double *>(c0->partials.p);
    const int ng = n;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_sc = carve(sizeof(CgScalars) * nsys);
    const size_t o_ex = carve(sizeof(double) * NEXTRA * nsys);
    const size_t o_ac = carve(sizeof(int32_t) * nsys);
    const size_t o_rs = carve(sizeof(int32_t) * nsys);
    const size_t o_hop = carve(sizeof(HopParams) * NHOP * ng);
    const size_t o_hring = carve(sizeof(HopParams) * 2 * RING_MAX * ng);
    const size_t o_vec = carve(sizeof(VecSys) * NVEC * nsys);
    const size_t o_pre = carve(sizeof(int64_t) * NHOP * (ng + 1));
    const size_t o_coef = carve(sizeof(OpCoeffs) * ng);
    const size_t o_hist = carve(sizeof(double) * 2 * HIST_MAX * nsys);
    CK(c0->scalars.ensure((int64_t)off));
    char *base = static_cast<char *>(c0->scalars.p);
    sc = reinterpret_cast<CgScalars *>(base + o_sc);
    extra = reinterpret_cast<double *>(base + o_ex);
    active = reinterpret_cast<int32_t *>(base + o_ac);
    restart = reinterpret_cast<int32_t *>(base + o_rs);
    hop_tab = reinterpret_cast<HopParams *>(base + o_hop);
    hop_ring_tab = reinterpret_cast<HopParams *>(base + o_hring);
    vec_tab = reinterpret_cast<VecSys *>(base + o_vec);
    prefix = reinterpret_cast<int64_t *>(base + o_pre);
    OpCoeffs *coef = reinterpret_cast<OpCoeffs *>(base + o_coef);
    std::vector<OpCoeffs> h_coef(ng);
    for (int j = 0; j < ng; ++j) h_coef[j] = groups[j].ctx->c;

    // descriptor tables
    h_hop.assign((size_t)NHOP * ng, HopParams{});
    h_prefix.assign((size_t)NHOP * (ng + 1), 0);
    for (int pid = 0; pid < NHOP; ++pid) {
        int64_t acc = 0;
        hop_lds[pid] = 0;
        for (int j = 0; j < ng; ++j) {
            const Group &g = groups[j];
            const HopParams h = make_hop_params(g.ctx->g, g.ctx->c, hop_links(g.ctx, hp[pid].prec, hp[pid].dag),
                                                static_cast<const int32_t *>(g.ctx->nbr.p),
                                                hop_args_for(g, hp[pid]));
            h_hop[(size_t)pid * ng + j] = h;
            h_prefix[(size_t)pid * (ng + 1) + j] = acc;
            acc += h.nblocks;
            if (h.stage_links) hop_lds[pid] = 1;  // sized below, once the loop variant is known
        }
        h_prefix[(size_t)pid * (ng + 1) + ng] = acc;
    }
    // groups of one batch launch must agree on staging (one dynamic LDS size)
    for (int pid = 0; pid < NHOP; ++pid)
        for (int j = 0; j < ng; ++j) h_hop[(size_t)pid * ng + j].stage_links = hop_lds[pid] > 0 &&
            h_hop[(size_t)pid * ng + j].stage_links;
    // one batched launch runs one loop variant for every group: that of the
    // group with the most site blocks (the one its tuning was measured for
    // matters most), the matrix-core one only if every group can run it
    for (int pid = 0; pid < NHOP; ++pid) {
        bool all_mf = true;
        int big = 0;
        for (int j = 0; j < ng; ++j) {
            all_mf = all_mf && h_hop[(size_t)pid * ng + j].pf == 3;
            if (h_hop[(size_t)pid * ng + j].nblocks > h_hop[(size_t)pid * ng + big].nblocks) big = j;
        }
        hop_pf[pid] = h_hop[(size_t)pid * ng + big].pf;
        if (hop_pf[pid] == 3 && !all_mf) hop_pf[pid] = 2;
        // dynamic LDS of the launch: the largest staged record block of its groups
        const bool rows = hop_pf[pid] == 3;
        hop_lds[pid] = 0;
        bool multi = false;
        for (int j = 0; j < ng; ++j) {
            if (h_hop[(size_t)pid * ng + j].stage_links)
                hop_lds[pid] = std::max(hop_lds[pid], hop_link_lds_bytes(hp[pid].prec, groups[j].ctx->g.Ls, rows));
            multi = multi || h_hop[(size_t)pid * ng + j].nrhs > 1;
        }
        // the I^-1 epilogue's buffer: over the links (one system per group)
        // or past them
        if (hp[pid].epi & EPI_M5INV) {
            const size_t off = multi ? hop_lds[pid] : 0;
            for (int j = 0; j < ng; ++j) h_hop[(size_t)pid * ng + j].m5_off = (int)off;
            hop_lds[pid] = std::max(hop_lds[pid], off + m5_epilogue_lds_bytes(hp[pid].prec));
        }
    }
    h_vec.assign((size_t)NVEC * nsys, VecSys{});
    for (const Group &g : groups)
        for (int r = 0; r < g.nrhs; ++r) {
            const int j = g.sys0 + r;
            auto F = [&](Field k) { return g.f[k] + r * g.fb[k]; };
            VecSys v{};
            v.N5 = g.ctx->g.N5;
            v.flag = j;
            v.Ls = g.ctx->g.Ls;
            v.coef = coef + (&g - groups.data());
            v.partials = part + (int64_t)j * pstride;
            v.nparts = g.blas_blocks;
            VecSys t = v;
            t = v; t.a = F(F_RH); t.b = F(F_R);
            h_vec[(size_t)VP_CONV_RH_R * nsys + j] = t;
            t = v; t.a = F(F_X); t.d = F(F_XH);
            h_vec[(size_t)VP_ACC * nsys + j] = t;
            t = v; t.a = F(F_B); t.b = F(F_Q64); t.s1 = &extra[j * NEXTRA + X_MINUS1]; t.d = F(F_RH);
            h_vec[(size_t)VP_RES * nsys + j] = t;
            t = v; t.nparts = g.hop_blocks;
            h_vec[(size_t)VP_HOPRED * nsys + j] = t;
            h_vec[(size_t)VP_BLASRED * nsys + j] = v;
            t = v; t.a = F(F_B);
            h_vec[(size_t)VP_NORM_B * nsys + j] = t;
            t = v; t.a = F(F_ETA_E);
            h_vec[(size_t)VP_NORM_EE * nsys + j] = t;
            t = v; t.a = F(F_ETA_O);
            h_vec[(size_t)VP_NORM_EO * nsys + j] = t;
            t = v; t.a = F(F_B); t.b = F(F_RH);
            h_vec[(size_t)VP_CONV_B_RH * nsys + j] = t;
            t = v; t.a = F(F_X); t.b = F(F_P); t.c = F(F_R); t.d = F(F_S); t.s0 = &sc[j].alpha;
            h_vec[(size_t)VP_XR_N * nsys + j] = t;
            t = v; t.a = F(F_R); t.b = F(F_P); t.d = F(F_P); t.s1 = &sc[j].beta;
            h_vec[(size_t)VP_PUPD_N * nsys + j] = t;
            t = v; t.a = F(F_B); t.b = F(F_PE); t.s1 = &extra[j * NEXTRA + X_MINUS1]; t.d = F(F_RH);
            h_vec[(size_t)VP_RES_N * nsys + j] = t;
            t = v; t.a = F(F_B); t.b = F(F_XH);
            h_vec[(size_t)VP_DOT_B_XH * nsys + j] = t;
            t = v; t.a = F(F_XH); t.b = F(F_XH); t.d = F(F_RH);
            h_vec[(size_t)VP_TWO_XH * nsys + j] = t;
            t = v; t.a = F(F_S); t.b = F(F_P); t.c = F(F_X); t.s0 = &sc[j].alpha; t.s1 = &sc[j].beta;
            h_vec[(size_t)VP_PUPD_X * nsys + j] = t;
            t = v; t.a = F(F_P); t.c = F(F_X); t.s0 = &sc[j].alpha;
            h_vec[(size_t)VP_XFLUSH * nsys + j] = t;
            t = v; t.a = F(F_S); t.b = g.pring + r * g.fb[F_P]; t.sstride = g.fb[F_P] * g.nrhs;
            t.s1 = &sc[j].beta;
            h_vec[(size_t)VP_PUPD_R * nsys + j] = t;
            t = v; t.b = g.pring + r * g.fb[F_P]; t.sstride = g.fb[F_P] * g.nrhs; t.c = F(F_X);
            t.s0 = &sc[j].aring[0];
            h_vec[(size_t)VP_XRING * nsys + j] = t;
            t = v; t.a = F(F_R); t.b = g.pring + r * g.fb[F_P]; t.sstride = g.fb[F_P] * g.nrhs;
            t.s1 = &sc[j].beta;
            h_vec[(size_t)VP_PUPD_RN * nsys + j] = t;
            t = v; t.c = F(F_R); t.d = F(F_S); t.s0 = &sc[j].alpha;
            h_vec[(size_t)VP_R_N * nsys + j] = t;
            t = v; t.a = F(F_R); t.b = F(F_Q); t.c = F(F_U); t.s0 = &sc[j].alpha; t.nparts = g.hop_blocks;
            h_vec[(size_t)VP_RUPD * nsys + j] = t;
            t = v; t.a = F(F_Q);
            h_vec[(size_t)VP_NORM_Q * nsys + j] = t;
            t = v; t.a = F(F_S);
            h_vec[(size_t)VP_NORM_S * nsys + j] = t;
            t = v; t.a = F(F_T64);
            h_vec[(size_t)VP_NORM_T64 * nsys + j] = t;
            t = v; t.a = F(F_Q64);
            h_vec[(size_t)VP_NORM_Q64 * nsys + j] = t;
        }
    h_active.assign(nsys, 1);
    h_restart.assign(nsys, 1);
    CK(hipMemcpyAsync(hop_tab, h_hop.data(), sizeof(HopParams) * h_hop.size(), hipMemcpyHostToDevice, st));
    if (ring > 1 && ng > 1) {
        // per slot: the same descriptors with every operand that is p moved to the slot
        h_hop_ring.assign((size_t)2 * ring * ng, HopParams{});
        for (int s = 0; s < ring; ++s)
            for (int j2 = 0; j2 < 2; ++j2) {
                const int pid = j2 == 0 ? HP_D0A : HP_D0B;
                for (int j = 0; j < ng; ++j) {
                    const Group &g = groups[j];
                    const char *ps = g.pring + (int64_t)s * g.fb[F_P] * g.nrhs;
                    HopParams h = h_hop[(size_t)pid * ng + j];
                    if (hp[pid].in == F_P) h.in = ps;
                    if (hp[pid].x == F_P) h.x = ps;
                    if (hp[pid].y == F_P) h.y = ps;
                    h_hop_ring[((size_t)s * 2 + j2) * ng + j] = h;
                }
            }
        CK(hipMemcpyAsync(hop_ring_tab, h_hop_ring.data(), sizeof(HopParams) * h_hop_ring.size(),
                          hipMemcpyHostToDevice, st));
    }
    CK(hipMemcpyAsync(vec_tab, h_vec.data(), sizeof(VecSys) * h_vec.size(), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(prefix, h_prefix.data(), sizeof(int64_t) * h_prefix.size(), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(coef, h_coef.data(), sizeof(OpCoeffs) * ng, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(active, h_active.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(restart, h_restart.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
    hist = reinterpret_cast<double *>(base + o_hist);
    std::vector<CgScalars> h_sc(nsys, CgScalars{});
    for (int j = 0; j < nsys; ++j) {
        h_sc[j].hist = hist + (size_t)2 * HIST_MAX * j;
        h_sc[j].nhist = 0;
        h_sc[j].hmax = HIST_MAX;
    }
    CK(hipMemcpyAsync(sc, h_sc.data(), sizeof(CgScalars) * nsys, hipMemcpyHostToDevice, st));
    std::vector<double> h_extra((size_t)nsys * NEXTRA, 0.0);
    for (int j = 0; j < nsys; ++j) h_extra[(size_t)j * NEXTRA + X_MINUS1] = -1.0;
    CK(hipMemcpyAsync(extra, h_extra.data(), sizeof(double) * h_extra.size(), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));  // the host tables above are pageable and local
    int dev = 0, ncu = 256;
    CK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 256;
    batch_grid = ncu * 8;
    return MOBIUS_OK;
}

HopArgs Batch::hop_args_for(const Group &g, const HopPattern &p) const
{
    HopArgs a;
    a.prec = p.prec;
    a.dag = p.dag;
    a.epi = p.epi;
    a.out_parity = p.out_parity;
    a.in = g.f[p.in];
    a.out = g.f[p.out];
    a.x = p.x == F_NONE ? nullptr : g.f[p.x];
    a.y = p.y == F_NONE ? nullptr : g.f[p.y];
    a.partials = p.norm ? part + (int64_t)g.sys0 * pstride : nullptr;
    a.nrhs = g.nrhs;
    a.active = active + g.sys0;
    a.fstride = g.fb[p.in];
    a.pstride = pstride;
    a.tune = &g.ctx->tune[p.prec];
    return a;
}

void Batch::acct_hop(int prec, int epi, double fields, double n5)
{
    // per active system: in + out (+ x, + y) spinors; links once per group
    double nf = 2 + ((epi & (EPI_PRESUB | EPI_POSTSUB)) ? 1 : 0) + ((epi & (EPI_M5ADD | EPI_M5SUB)) ? 1 : 0);
    abytes += nf * fields + sum_links(prec);
    aflops += n5 * (1416 + ((epi & EPI_M5INV) ? 96 : 0) + ((epi & (EPI_PRESUB | EPI_POSTSUB)) ? 24 : 0) +
                    ((epi & (EPI_M5ADD | EPI_M5SUB)) ? 96 : 0) + ((epi & EPI_NORM) ? 48 : 0));
}

hipError_t Batch::hop(int pid)
{
    const HopPattern &p = hp[pid];
    acct_hop(p.prec, p.epi, sum_fb(p.prec, true), sum_n5(true));
    if (p.norm && !fused_norm) {
        // the kernel without the fused sum, then |out|^2 of every active system
        HopPattern q = p;
        q.epi &= ~EPI_NORM;
        q.norm = false;
        const int npid = p.out == F_Q ? VP_NORM_Q : VP_NORM_S;
        if (!count_only) {
            hipError_t e = launch_pattern(q, pid);
            if (e != hipSuccess) return e;
        }
        return vec(npid, VEC_NORM2, p.prec, p.prec);
    }
    if (count_only) return hipSuccess;
    return launch_pattern(p, pid);
}

hipError_t Batch::launch_pattern(const HopPattern &p, int pid)
{
    if (ngroups() == 1) {
        const Group &g = groups[0];
        return launch_hop(g.ctx->g, g.ctx->c, hop_links(g.ctx, p.prec, p.dag),
                          static_cast<const int32_t *>(g.ctx->nbr.p), hop_args_for(g, p), st);
    }
    const HopParams *tab = hop_tab + (size_t)pid * ngroups();
    if (ring > 1 && (pid == HP_D0A || pid == HP_D0B))
        tab = hop_ring_tab + ((size_t)cur_slot * 2 + (pid == HP_D0B ? 1 : 0)) * ngroups();
    return launch_hop_batch(p.prec, p.dag, p.epi, tab, ngroups(), prefix + (size_t)pid * (ngroups() + 1),
                            hop_lds[pid], batch_grid, hop_pf[pid], st);
}

hipError_t Batch::hop_group(const Group &g, int prec, int dag, int epi, int out_parity, Field in,
                            Field out, Field x, Field y, bool norm)
{
    HopPattern p{prec, dag, epi, out_parity, in, out, x, y, norm};
    HopArgs a = hop_args_for(g, p);
    a.active = nullptr;  // every right-hand side of the group
    abytes += (2 + (x != F_NONE) + (y != F_NONE)) * (double)g.fb[in] * g.nrhs +
              72.0 * g.ctx->g.Vh * link_elem_bytes(prec);
    aflops += (double)g.ctx->g.N5 * g.nrhs * 1416;
    return launch_hop(g.ctx->g, g.ctx->c, hop_links(g.ctx, prec, dag),
                      static_cast<const int32_t *>(g.ctx->nbr.p), a, st);
}

hipError_t Batch::vec(int pid, int kind, int prec, int prec2, bool all)
{
    const double fb = sum_fb(prec, true), fb2 = sum_fb(prec2, true), n5 = sum_n5(true);
    switch (kind) {
    case VEC_CG_XR:
        if (pid == VP_R_N) {  // r -= alpha s only
            abytes += 3 * fb;
            aflops += 96 * n5;
        } else {
            abytes += 2 * fb2 + 4 * fb;
            aflops += 144 * n5;
        }
        break;
    case VEC_AXPBY: abytes += 3 * fb; aflops += 48 * n5; break;
    case VEC_AXPBY_NORM: abytes += 3 * fb; aflops += 96 * n5; break;
    case VEC_NORM2: abytes += fb; aflops += 48 * n5; break;
    case VEC_CONVERT: abytes += fb + fb2; break;
    case VEC_ACCUMULATE: abytes += 2 * fb + 2 * sum_fb(MOBIUS_F64, true); aflops += 24 * n5; break;
    case VEC_DOT: abytes += 2 * fb; aflops += 48 * n5; break;
    // x (prec2) += alpha p, p = s + beta p: reads s, p, x; writes p, x
    case VEC_PUPD_X: abytes += 3 * fb + 2 * fb2; aflops += 96 * n5; break;
    // x (prec2) += alpha p: reads p, x; writes x
    case VEC_XFLUSH: abytes += fb + 2 * fb2; aflops += 48 * n5; break;
    }
    if (count_only) return hipSuccess;
    return launch_vec_batch(kind, prec, prec2, vec_tab + (size_t)pid * nsys, nsys, max_n5,
                            all ? nullptr : active, st);
}

// p[slot] = s + beta p[prev] (kind VEC_PUPD_RING: reads s and p[prev], writes
// p[slot]) or x += sum_{i < a0} alpha_i p[i] (VEC_XRING: reads a0 directions
// and x, writes x)
hipError_t Batch::ring_vec(int pid, int kind, int a0, int a1)
{
    const double fb = sum_fb(lo, true), fb2 = sum_fb(px, true), n5 = sum_n5(true);
    if (kind == VEC_PUPD_RING) {
        abytes += 3 * fb;
        aflops += 48 * n5;
    } else {
        abytes += a0 * fb + 2 * fb2;
        aflops += 48.0 * a0 * n5;
    }
    if (count_only) return hipSuccess;
    return launch_ring_batch(kind, lo, px, vec_tab + (size_t)pid * nsys, nsys, max_n5, active, a0, a1,
                             st);
}

hipError_t Batch::reduce(int pid, double *out, int64_t stride, bool all)
{
    if (count_only) return hipSuccess;
    return launch_reduce_batch(vec_tab + (size_t)pid * nsys, nsys, all ? nullptr : active, 0, out,
                               stride, st);
}

hipError_t Batch::next_u(bool only_active)
{
    if (form == FORM_RIGHT || form == FORM_PLAIN) return hipSuccess;  // their A^+ starts from r itself
    if (form == FORM_LHAT) {  // u = B^+ I^-+ r, through t
        hipError_t e = m5inv_all(lo, 1, F_R, F_T, only_active);
        if (e != hipSuccess) return e;
        return m5inv_all(lo, 1, F_T, F_U, only_active, true);
    }
    return m5inv_all(lo, form == FORM_LEFT ? 1 : 0, F_R, F_U, only_active);
}

hipError_t Batch::psi_odd()
{
    if (form != FORM_RIGHT && form != FORM_LHAT) return hipSuccess;
    for (const Group &g : groups) {
        abytes += 2.0 * g.fb[F_XH] * g.nrhs;
        aflops += 96.0 * g.ctx->g.N5 * g.nrhs;
        // right: psi_o = I^-1 z; left form of D^: psi_o = B^-1 y
        const OpCoeffs c = form == FORM_RIGHT ? g.ctx->c : b_coeffs(g.ctx->c, g.ctx->g.Ls);
        hipError_t e = launch_m5(g.ctx->g, c, MOBIUS_F64, 1, 0, g.f[F_XH], g.f[F_PO], g.nrhs, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// out = I^-1 in (I^-+ for dag), or with bmix B in (B^+ in) -- the left form's
// s-direction factor, through the same kernel with B's coefficients
hipError_t Batch::m5inv_all(int prec, int dag, Field in, Field out, bool only_active, bool bmix)
{
    for (const Group &g : groups) {
        for (int r = 0; r < g.nrhs; ++r) {
            // eager callers skip the systems that are off (a reliable update
            // leaves the Krylov vectors of the systems sitting it out as they are)
            if (only_active && !h_active[g.sys0 + r]) continue;
            abytes += 2.0 * g.fb[in];
            aflops += 96.0 * g.ctx->g.N5;
            if (count_only) continue;
            hipError_t e = bmix ? launch_m5(g.ctx->g, b_coeffs(g.ctx->c, g.ctx->g.Ls), prec, 0, dag,
                                            g.f[in] + r * g.fb[in], g.f[out] + r * g.fb[out], 1, st)
                                : launch_m5(g.ctx->g, g.ctx->c, prec, 1, dag, g.f[in] + r * g.fb[in],
                                            g.f[out] + r * g.fb[out], 1, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

constexpr int64_t SC_STRIDE = sizeof(CgScalars) / sizeof(double);

// s = D^+ r (gamma_new); beta; p = s + beta p;  q = D p (qq); alpha;  x += alpha p, r -= alpha q (rr)
// (with a ring of directions, x += sum alpha p once at the end of the chunk)
hipError_t Batch::body(int q, int k)
{
    hipError_t e;
    dirac += 4;
    if ((e = hop(HP_D1B)) != hipSuccess) return e;
    if ((e = hop(HP_D1C)) != hipSuccess) return e;
    if ((e = reduce(norm_red(), &sc[0].gamma_new, SC_STRIDE)) != hipSuccess) return e;
    if (!count_only && (e = launch_cg_scalar_batch(sc, nsys, 1, active, restart, st)) != hipSuccess) return e;
    const int slot = ring > 1 ? q : -1;
    if (ring > 1) {
        cur_slot = slot;
        for (Group &g : groups) g.f[F_P] = g.pring + (int64_t)slot * g.fb[F_P] * g.nrhs;
        if ((e = ring_vec(VP_PUPD_R, VEC_PUPD_RING, slot, q == 0 ? ring - 1 : q - 1)) != hipSuccess)
            return e;
    } else if ((e = vec(VP_PUPD_X, VEC_PUPD_X, lo, px)) != hipSuccess) {
        return e;
    }
    if (form == FORM_RIGHT && (e = m5inv_all(lo, 0, F_P, F_U)) != hipSuccess) return e;  // v = I^-1 p
    if ((e = hop(HP_D0A)) != hipSuccess) return e;
    if ((e = hop(HP_D0B)) != hipSuccess) return e;
    if ((e = reduce(norm_red(), &sc[0].qq, SC_STRIDE)) != hipSuccess) return e;
    if (!count_only && (e = launch_cg_scalar_batch(sc, nsys, 0, active, restart, st, slot)) != hipSuccess)
        return e;
    if ((e = rupd()) != hipSuccess) return e;
    if ((e = reduce(VP_RUPD, &sc[0].rr, SC_STRIDE)) != hipSuccess) return e;
    if (ring > 1 && q == k - 1) return ring_vec(VP_XRING, VEC_XRING, k, 0);
    return hipSuccess;
}

// Normal equations, p = r + beta p;  q = D p (|q|^2 -> alpha);  s = D^+ q;
// x += alpha p, r -= alpha s (|r|^2 -> the next gamma); with a ring of
// directions, x += sum alpha p once at the end of the chunk.
hipError_t Batch::body_normal(int q, int k)
{
    hipError_t e;
    dirac += 4;
    if (!count_only && (e = launch_cg_scalar_batch(sc, nsys, 1, active, restart, st)) != hipSuccess) return e;
    const int slot = ring > 1 ? q : -1;
    if (ring > 1) {
        cur_slot = slot;
        for (Group &g : groups) g.f[F_P] = g.pring + (int64_t)slot * g.fb[F_P] * g.nrhs;
        if ((e = ring_vec(VP_PUPD_RN, VEC_PUPD_RING, slot, q == 0 ? ring - 1 : q - 1)) != hipSuccess)
            return e;
    } else if ((e = vec(VP_PUPD_N, VEC_AXPBY, lo, lo)) != hipSuccess) {
        return e;
    }
    if ((e = hop(HP_D0A)) != hipSuccess) return e;
    if ((e = hop(HP_D0B)) != hipSuccess) return e;
    if ((e = reduce(norm_red(), &sc[0].qq, SC_STRIDE)) != hipSuccess) return e;
    if (!count_only && (e = launch_cg_scalar_batch(sc, nsys, 0, active, restart, st, slot)) != hipSuccess)
        return e;
    if ((e = m5inv_dag_all(lo, F_Q, F_U)) != hipSuccess) return e;
    if ((e = hop(HP_D1B)) != hipSuccess) return e;
    if ((e = hop(HP_D1Q)) != hipSuccess) return e;
    if ((e = vec(ring > 1 ? VP_R_N : VP_XR_N, VEC_CG_XR, lo, px)) != hipSuccess) return e;
    if ((e = reduce(VP_BLASRED, &sc[0].rr, SC_STRIDE)) != hipSuccess) return e;
    if ((e = reduce(VP_BLASRED, &sc[0].gamma_new, SC_STRIDE)) != hipSuccess) return e;
    if (ring > 1 && q == k - 1) return ring_vec(VP_XRING, VEC_XRING, k, 0);
    return hipSuccess;
}

hipError_t Batch::rupd()
{
    const double fb = sum_fb(lo, true), n5 = sum_n5(true);
    const int mode = rupd_mode();
    abytes += (mode == 2 ? 3 : 4) * fb;
    aflops += (48 + (mode == 2 ? 0 : 96) + (mode == 3 ? 48 : 0) + 48) * n5;
    if (count_only) return hipSuccess;
    return launch_rupd_m5inv_batch(lo, vec_tab + (size_t)VP_RUPD * nsys, nsys, max_site_blocks, active,
                                   mode, st);
}

hipError_t Batch::reliable_update()
{
    hipError_t e;
    dirac += normal ? 4 : 2;
    if (!normal && ring == 1) {  // the last alpha p of the iteration, then no pending update
        if ((e = vec(VP_XFLUSH, VEC_XFLUSH, lo, px)) != hipSuccess) return e;
        if ((e = launch_cg_scalar_batch(sc, nsys, 2, active, restart, st)) != hipSuccess) return e;
    }
    if ((e = vec(VP_ACC, VEC_ACCUMULATE, px, MOBIUS_F64)) != hipSuccess) return e;
    if (form == FORM_RIGHT && (e = m5inv_all(MOBIUS_F64, 0, F_XH, F_U64, true)) != hipSuccess) return e;
    if ((e = hop(HP_H0A)) != hipSuccess) return e;
    if ((e = hop(HP_H0B)) != hipSuccess) return e;
    if (normal) {  // r = b - D^+ D x_hi
        if ((e = m5inv_dag_all(MOBIUS_F64, F_Q64, F_U64, true)) != hipSuccess) return e;
        if ((e = hop(HP_N64B)) != hipSuccess) return e;
        if ((e = hop(HP_N64C)) != hipSuccess) return e;
        if ((e = vec(VP_RES_N, VEC_AXPBY_NORM, MOBIUS_F64, MOBIUS_F64)) != hipSuccess) return e;
        if ((e = reduce(VP_BLASRED, &extra[X_HR], NEXTRA)) != hipSuccess) return e;
        if ((e = reduce(VP_BLASRED, &sc[0].gamma_new, SC_STRIDE)) != hipSuccess) return e;
    } else {
        if ((e = vec(VP_RES, VEC_AXPBY_NORM, MOBIUS_F64, MOBIUS_F64)) != hipSuccess) return e;
        if ((e = reduce(VP_BLASRED, &extra[X_HR], NEXTRA)) != hipSuccess) return e;
    }
    if ((e = vec(VP_CONV_RH_R, VEC_CONVERT, MOBIUS_F64, lo)) != hipSuccess) return e;
    return normal ? hipSuccess : next_u(true);  // the solve of r the next step starts from
}

// psi_e = I^-1 (eta_e - D_eo x_hi); |eta - D_DW psi|^2 per parity -> extra
hipError_t Batch::finalize_group(const Group &g)
{
    hipError_t e;
    dirac += 3;
    const bool fuse = g.nrhs == 1;
    const int nepi = fuse ? EPI_NORM : 0;
    // partial sums of this group's systems: from the hop (fused) or a norm pass
    auto norms = [&](int npid, Extra slot) -> hipError_t {
        if (!fuse) {
            abytes += (double)g.fb[F_T64] * g.nrhs;
            hipError_t x = launch_vec_batch(VEC_NORM2, MOBIUS_F64, MOBIUS_F64,
                                            vec_tab + (size_t)npid * nsys + g.sys0, g.nrhs,
                                            g.ctx->g.N5, nullptr, st);
            if (x != hipSuccess) return x;
        }
        return launch_reduce_batch(vec_tab + (size_t)(fuse ? VP_HOPRED : VP_BLASRED) * nsys + g.sys0,
                                   g.nrhs, nullptr, 0, &extra[g.sys0 * NEXTRA + slot], NEXTRA, st);
    };
    // psi_e = I^-1 (eta_e - D_eo psi_o) (the adjoint system: its own blocks),
    // then eta - D psi on both parities
    const int dg = adj() ? 1 : 0;
    const Field po = psi_o();
    if ((e = hop_group(g, MOBIUS_F64, dg, EPI_PRESUB | EPI_M5INV, 0, po, F_PE, F_ETA_E, F_NONE, false)) != hipSuccess) return e;
    if ((e = hop_group(g, MOBIUS_F64, dg, EPI_M5ADD | EPI_PRESUB | nepi, 0, po, F_T64, F_ETA_E, F_PE, fuse)) != hipSuccess) return e;
    if ((e = norms(VP_NORM_T64, X_RES_E)) != hipSuccess) return e;
    if ((e = hop_group(g, MOBIUS_F64, dg, EPI_M5ADD | EPI_PRESUB | nepi, 1, F_PE, F_Q64, F_ETA_O, po, fuse)) != hipSuccess) return e;
    return norms(VP_NORM_Q64, X_RES_O);
}

// which: -1 = rr of every system, otherwise extra[which] of every system
int Batch::fetch(std::vector<double> &out, int which)
{
    out.resize(nsys);
    if (which < 0) {
        std::vector<CgScalars> h(nsys);
        CK(hipMemcpyAsync(h.data(), sc, sizeof(CgScalars) * nsys, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int j = 0; j < nsys; ++j) out[j] = h[j].rr;
    } else {
        std::vector<double> h((size_t)nsys * NEXTRA);
        CK(hipMemcpyAsync(h.data(), extra, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int j = 0; j < nsys; ++j) out[j] = h[(size_t)j * NEXTRA + which];
    }
    return MOBIUS_OK;
}

// Eigenvalue bounds of a symmetric tridiagonal matrix (diagonal d, off-diagonal
// e[k] between k-1 and k, e[0] unused): the smallest and the largest, by
// bisection on the Sturm count (number of eigenvalues below x).
static void tridiag_extremes(const std::vector<double> &d, const std::vector<double> &e,
                             double &lmin, double &lmax)
{
    const size_t n = d.size();
    double lo = INFINITY, hi = -INFINITY;
    for (size_t k = 0; k < n; ++k) {  // Gershgorin
        const double r = (k > 0 ? std::fabs(e[k]) : 0.0) + (k + 1 < n ? std::fabs(e[k + 1]) : 0.0);
        lo = std::min(lo, d[k] - r);
        hi = std::max(hi, d[k] + r);
    }
    auto below = [&](double x) {
        size_t c = 0;
        double q = 1.0;
        for (size_t k = 0; k < n; ++k) {
            q = d[k] - x - (k > 0 ? e[k] * e[k] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            c += q < 0.0;
        }
        return c;
    };
    auto kth = [&](size_t want) {  // the eigenvalue with `want` eigenvalues below it
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
            const double m = 0.5 * (a + b);
            if (below(m) > want) b = m; else a = m;
        }
        return 0.5 * (a + b);
    };
    lmin = kth(0);
    lmax = kth(n - 1);
}

// cond(D_pre) = sqrt(lambda_max / lambda_min) of the normal operator, from the
// Lanczos tridiagonal that the CG coefficients define:
//   T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},  T_{k-1,k} = sqrt(beta_{k-1})/alpha_{k-1}
// (beta = 0 where a Krylov segment restarts: T is then block diagonal and its
// extreme eigenvalues are the extremes over the segments).  0 when no
// iteration ran.
int Batch::kappa(std::vector<double> &out)
{
    out.assign(nsys, 0.0);
    std::vector<CgScalars> h(nsys);
    CK(hipMemcpyAsync(h.data(), sc, sizeof(CgScalars) * nsys, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    std::vector<double> hb;
    for (int j = 0; j < nsys; ++j) {
        const int64_t n = h[j].nhist;
        if (n < 1) continue;
        hb.resize(2 * n);
        CK(hipMemcpy(hb.data(), h[j].hist, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
        std::vector<double> d, e;
        double prev_a = 0;
        for (int64_t k = 0; k < n; ++k) {
            const double b = hb[2 * k], a = hb[2 * k + 1];
            if (!(a > 0) || !std::isfinite(a)) break;
            const bool link = !d.empty() && b > 0 && prev_a > 0;
            d.push_back(1.0 / a + (link ? b / prev_a : 0.0));
            e.push_back(link ? std::sqrt(b) / prev_a : 0.0);
            prev_a = a;
        }
        if (d.empty()) continue;
        double lmin, lmax;
        tridiag_extremes(d, e, lmin, lmax);
        out[j] = lmin > 0 ? std::sqrt(lmax / lmin) : INFINITY;
    }
    return MOBIUS_OK;
}

// The derivative pass of the pseudofermion action after the normal-equations
// solve (one system, x_hi = X):
//   Z = I^-1 D_eo X (even), Y = D_pre X, Yt = I^-+ Y, W = I^-+ (D_oe)^+ Yt (even),
//   link gradient per parity from (L, R) = (Yt, X) on odd and (W, Z) on even sites,
//   S = Re <phi_o, X>,  dS/dphi = 2 X.
int force_pass(Batch &B, ForceOut &fo)
{
    const Group &g = B.groups[0];
    const Geometry &G = g.ctx->g;
    const int32_t *nbr = static_cast<const int32_t *>(g.ctx->nbr.p);
    hipStream_t st = B.st;
    if (fo.grad_links) {  // the link derivative (skipped when no link gradient is asked for)
        B.dirac += 3;
        CK(B.hop_group(g, MOBIUS_F64, 0, EPI_M5INV, 0, F_XH, F_PE, F_NONE, F_NONE, false));
        CK(B.hop_group(g, MOBIUS_F64, 0, EPI_M5INV | EPI_POSTSUB, 1, F_PE, F_Q64, F_XH, F_NONE, false));
        CK(launch_m5(G, g.ctx->c, MOBIUS_F64, 1, 1, g.f[F_Q64], g.f[F_U64], 1, st));
        CK(B.hop_group(g, MOBIUS_F64, 1, EPI_M5INV, 0, F_U64, F_T64, F_NONE, F_NONE, false));
        CK(launch_force(G, g.ctx->c, 1, nbr, g.f[F_U64], g.f[F_XH], g.f[F_T64], g.f[F_PE], fo.grad_links, st,
                        1.0, false, g.ctx->P.mu));
        CK(launch_force(G, g.ctx->c, 0, nbr, g.f[F_T64], g.f[F_PE], g.f[F_U64], g.f[F_XH], fo.grad_links, st,
                        1.0, false, g.ctx->P.mu));
        B.abytes += 2.0 * 4 * g.fb[F_XH] + 4.0 * G.V * 9 * 16;
        B.aflops += 2.0 * G.N5 * 4 * (2 * 24 + 2 * 2 * 9 * 8 + 96);
    }
    CK(B.vec(VP_DOT_B_XH, VEC_DOT, MOBIUS_F64, MOBIUS_F64, true));
    CK(B.reduce(VP_BLASRED, &B.extra[X_ACTION], NEXTRA, true));
    CK(B.vec(VP_TWO_XH, VEC_AXPBY, MOBIUS_F64, MOBIUS_F64, true));
    CK(launch_zero(g.f[F_ETA_E], g.fb[F_ETA_E], st));
    CK(launch_unpack_spinor(G, MOBIUS_F64, g.f[F_ETA_E], g.f[F_RH], fo.grad_phi, 1, st));
    B.abytes += 2.0 * G.N5 * 12 * 16 + 2.0 * g.fb[F_XH];
    std::vector<double> S;
    if (int rc = B.fetch(S, X_ACTION)) return rc;
    fo.action = S[0];
    return MOBIUS_OK;
}

int run(mobius_ctx *const *ctxs, int ngroups, const void *const *src, void *const *sol,
        const mobius_solve_opts &o, mobius_solve_info *info, hipStream_t user, ForceOut *fo,
        int form)
{
    const int nrhs = o.nrhs > 0 ? o.nrhs : 1;
    const double tol = o.tol > 0 ? o.tol : 1e-10;
    const double err_tol = o.err_tol > 0 ? o.err_tol : 0.0;
    const int maxiter = o.maxiter > 0 ? o.maxiter : 10000;
    const bool mixed = o.inner_prec != MOBIUS_F64;
    // Default update threshold per operator precision.  The binary16 Krylov
    // vectors drift from the true residual after about half a decade of
    // reduction, so the FP16 operator updates every factor 0.3 (at 24^3 x 64,
    // Ls = 12 this took 1256 iterations against 1704 at 0.1; 16^3 x 32, Ls = 16
    // point sources 1120 against ~1700); the FP32 iteration count does not
    // depend on it.
    const double delta_default = o.inner_prec == MOBIUS_F16 ? 0.3 : 0.1;
    const double delta = mixed ? (o.reliable_delta > 0 ? o.reliable_delta : delta_default) : 0.0;
    const int check = o.check_every > 0 ? o.check_every : (mixed ? 8 : 16);
    const bool use_graph = env_int("MOBIUS_GRAPH", 1) != 0;

    Batch B;
    mobius_ctx *c0 = ctxs[0];
    if (!c0->solve_stream) CK(hipStreamCreateWithFlags(&c0->solve_stream, hipStreamNonBlocking));
    B.st = c0->solve_stream;
    // events and the captured graph are released on every return path
    struct Owned {
        hipEvent_t ev_in = nullptr, ev0 = nullptr, ev1 = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        ~Owned()
        {
            if (gexec) (void)hipGraphExecDestroy(gexec);
            if (graph) (void)hipGraphDestroy(graph);
            for (hipEvent_t e : {ev_in, ev0, ev1})
                if (e) (void)hipEventDestroy(e);
        }
    } own;
    CK(hipEventCreateWithFlags(&own.ev_in, hipEventDisableTiming));
    CK(hipEventCreate(&own.ev0));
    CK(hipEventCreate(&own.ev1));
    CK(hipEventRecord(own.ev_in, user));
    CK(hipStreamWaitEvent(B.st, own.ev_in, 0));
    CK(hipEventRecord(own.ev0, B.st));
    B.normal = fo != nullptr;
    B.form = form;
    // the deferred x update: CG with a lower-precision inner operator (the FP32
    // x against FP32 or binary16 directions), one slot per iteration of a
    // chunk; MOBIUS_DEFER_X=0 updates x in every iteration
    if (mixed && check >= 2 && check <= RING_MAX && env_int("MOBIUS_DEFER_X", 1) != 0)
        B.ring = check;


    if (int rc = B.setup(ctxs, ngroups, src, sol, nrhs, o.inner_prec)) return rc;
    const int nsys = B.nsys;
    hipStream_t st = B.st;

    // source preparation, per group: b' = I^-1 (eta_o - D_oe I^-1 eta_e), or
    // for the normal equations b = the odd half of the source
    for (const Group &g : B.groups) {
        const double canon = 2.0 * g.ctx->g.N5 * 12 * 16 * g.nrhs;
        B.abytes += canon + 2.0 * g.fb[F_ETA_E] * g.nrhs;
        if (B.normal) {
            CK(launch_pack_spinor(g.ctx->g, MOBIUS_F64, g.src, g.f[F_ETA_E], g.f[F_B], g.nrhs, st));
            CK(launch_zero(g.f[F_ETA_O], g.fb[F_ETA_O] * g.nrhs, st));
        } else {
            // left: b' = I^-1 (eta_o - D_oe I^-1 eta_e); right and plain: b_R = eta_o - D_oe I^-1 eta_e;
            // adjoint system: b' = I^-+ (eta_o - (D^+)_oe I^-+ eta_e)
            const int dg = B.adj() ? 1 : 0;
            CK(launch_pack_spinor(g.ctx->g, MOBIUS_F64, g.src, g.f[F_ETA_E], g.f[F_ETA_O], g.nrhs, st));
            CK(launch_m5(g.ctx->g, g.ctx->c, MOBIUS_F64, 1, dg, g.f[F_ETA_E], g.f[F_T64], g.nrhs, st));
            const bool unprec = B.form == FORM_RIGHT || B.form == FORM_PLAIN;
            CK(B.hop_group(g, MOBIUS_F64, dg, unprec ? EPI_POSTSUB : EPI_PRESUB | EPI_M5INV, 1,
                           F_T64, B.form == FORM_LHAT ? F_Q64 : F_B, F_ETA_O, F_NONE, false));
            if (B.form == FORM_LHAT) {  // left form of D^: b^ = B b'
                B.abytes += 2.0 * g.fb[F_B] * g.nrhs;
                CK(launch_m5(g.ctx->g, b_coeffs(g.ctx->c, g.ctx->g.Ls), MOBIUS_F64, 0, 0, g.f[F_Q64], g.f[F_B],
                             g.nrhs, st));
            }
            B.dirac += 1;
        }
        CK(launch_zero(g.f[F_XH], g.fb[F_XH] * g.nrhs, st));
        CK(launch_zero(g.f[F_X], g.fb[F_X] * g.nrhs, st));
        // beta = 0 times p must be 0 (every slot of the ring)
        CK(launch_zero(g.pring, g.fb[F_P] * g.nrhs * B.ring, st));
    }
    CK(B.vec(VP_NORM_B, VEC_NORM2, MOBIUS_F64, MOBIUS_F64));
    CK(B.reduce(VP_BLASRED, &B.extra[X_BNORM2], NEXTRA, true));
    if (B.normal) CK(B.reduce(VP_BLASRED, &B.sc[0].gamma_new, SC_STRIDE, true));
    CK(B.vec(VP_NORM_EE, VEC_NORM2, MOBIUS_F64, MOBIUS_F64));
    CK(B.reduce(VP_BLASRED, &B.extra[X_ETA_E2], NEXTRA, true));
    CK(B.vec(VP_NORM_EO, VEC_NORM2, MOBIUS_F64, MOBIUS_F64));
    CK(B.reduce(VP_BLASRED, &B.extra[X_ETA_O2], NEXTRA, true));
    CK(B.vec(VP_CONV_B_RH, VEC_CONVERT, MOBIUS_F64, MOBIUS_F64));
    CK(B.vec(VP_CONV_RH_R, VEC_CONVERT, MOBIUS_F64, B.lo));
    if (!B.normal) {  // the iteration starts from the solve of r (left: u = I^-+ r) and no pending x update
        CK(B.next_u(false));
        CK(launch_cg_scalar_batch(B.sc, nsys, 2, nullptr, nullptr, st));
    }
    std::vector<double> bnorm2, eta_e2, eta_o2;
    if (int rc = B.fetch(bnorm2, X_BNORM2)) return rc;
    if (int rc = B.fetch(eta_e2, X_ETA_E2)) return rc;
    if (int rc = B.fetch(eta_o2, X_ETA_O2)) return rc;

    std::vector<double> tol_s(nsys, tol), rmax2(bnorm2), true_res(nsys, INFINITY),
        schur_res(nsys, INFINITY);
    std::vector<int> iters(nsys, 0), reliable(nsys, 0), converged(nsys, 0), pending(nsys, 0);
    for (int j = 0; j < nsys; ++j) {
        if (bnorm2[j] == 0.0) {  // nothing to iterate: psi_o = 0
            B.h_active[j] = 0;
            pending[j] = 1;
        }
    }

    hipGraphExec_t &gexec = own.gexec;
    hipGraph_t &graph = own.graph;
    int it = 0;
    auto sync_flags = [&]() -> int {
        CK(hipMemcpyAsync(B.active, B.h_active.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(B.restart, B.h_restart.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
        CK(hipStreamSynchronize(st));  // host copies are pageable; the device clears restart flags
        std::fill(B.h_restart.begin(), B.h_restart.end(), 0);
        return MOBIUS_OK;
    };
    if (int rc = sync_flags()) return rc;

    while (true) {
        // finalize systems whose Schur residual reached the target
        bool any_pending = false;
        for (int j = 0; j < nsys; ++j) any_pending |= pending[j] != 0;
        if (any_pending) {
            if (!B.normal) CK(B.psi_odd());
            for (const Group &g : B.groups) {
                bool gp = false;
                for (int r = 0; r < g.nrhs; ++r) gp |= pending[g.sys0 + r] != 0;
                if (gp && !B.normal) CK(B.finalize_group(g));
            }
            std::vector<double> re, ro, hr, kap;
            if (int rc = B.fetch(re, X_RES_E)) return rc;
            if (int rc = B.fetch(ro, X_RES_O)) return rc;
            if (int rc = B.fetch(hr, X_HR)) return rc;
            if (err_tol > 0)
                if (int rc = B.kappa(kap)) return rc;
            for (int j = 0; j < nsys; ++j) {
                if (!pending[j]) continue;
                pending[j] = 0;
                const double en = std::sqrt(eta_e2[j] + eta_o2[j]);
                schur_res[j] = bnorm2[j] > 0 ? std::sqrt(hr[j] / bnorm2[j]) : 0.0;
                if (B.normal)  // |b - D^+ D x| / |b| is the residual of the system itself
                    true_res[j] = schur_res[j];
                else
                    true_res[j] = en > 0 ? std::sqrt(re[j] + ro[j]) / en : 0.0;
                // bound on the relative error of the iterated unknown: cond(D_pre)
                // times the Schur residual (cond(D_pre)^2 for the normal equations)
                const double bound = err_tol > 0 ? (B.normal ? kap[j] * kap[j] : kap[j]) * schur_res[j] : 0.0;
                if (bnorm2[j] == 0.0 || (true_res[j] <= tol && bound <= err_tol)) {
                    converged[j] = 1;
                    B.h_active[j] = 0;
                } else {
                    const double f = true_res[j] > tol ? tol / true_res[j] : err_tol / bound;
                    tol_s[j] *= std::max(0.05, 0.5 * f);
                    B.h_active[j] = 1;
                    B.h_restart[j] = 1;
                }
            }
            if (int rc = sync_flags()) return rc;
        }
        if (B.nactive() == 0 || it >= maxiter) break;

        // a chunk of iterations
        const int k = std::min(check, maxiter - it);
        if (use_graph && k == check) {
            if (!gexec) {
                CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                hipError_t e = hipSuccess;
                for (int q = 0; q < k && e == hipSuccess; ++q) e = B.normal ? B.body_normal(q, k) : B.body(q, k);
                hipError_t e2 = hipStreamEndCapture(st, &graph);
                CK(e);
                CK(e2);
                CK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            } else {
                // account the replay without launching anything
                B.count_only = true;
                for (int q = 0; q < k; ++q) (void)(B.normal ? B.body_normal(q, k) : B.body(q, k));
                B.count_only = false;
            }
            CK(hipGraphLaunch(gexec, st));
        } else {
            // (a chunk shorter than check is the last one: it reaches maxiter)
            for (int q = 0; q < k; ++q) CK(B.normal ? B.body_normal(q, k) : B.body(q, k));
        }
        it += k;
        for (int j = 0; j < nsys; ++j)
            if (B.h_active[j]) iters[j] += k;

        std::vector<double> rr;
        if (int rc = B.fetch(rr, -1)) return rc;
        bool need_update = false;
        std::vector<int> upd(nsys, 0);
        for (int j = 0; j < nsys; ++j) {
            if (!B.h_active[j]) continue;
            if (!std::isfinite(rr[j]))
                return set_error(MOBIUS_EHIP, "CG breakdown: non-finite residual in system " +
                                                  std::to_string(j) + " after iteration " +
                                                  std::to_string(it));
            if (rr[j] <= tol_s[j] * tol_s[j] * bnorm2[j] || it >= maxiter ||
                (mixed && rr[j] < delta * delta * rmax2[j])) {
                upd[j] = 1;
                need_update = true;
            }
        }
        if (!need_update) continue;
        // reliable update of the systems that reached their own threshold; the
        // others sit it out (inactive for its kernels): an update forced on a
        // system whose residual has barely moved would restart its direction
        std::vector<int> sat_out(nsys, 0);
        bool any_out = false;
        for (int j = 0; j < nsys; ++j)
            if (B.h_active[j] && !upd[j]) {
                sat_out[j] = 1;
                B.h_active[j] = 0;
                any_out = true;
            }
        if (any_out) {
            CK(hipMemcpyAsync(B.active, B.h_active.data(), sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
            CK(hipStreamSynchronize(st));  // pageable host copy
        }
        CK(B.reliable_update());
        std::vector<double> hr;
        if (int rc = B.fetch(hr, X_HR)) return rc;
        for (int j = 0; j < nsys; ++j)
            if (sat_out[j]) B.h_active[j] = 1;
        for (int j = 0; j < nsys; ++j) {
            if (!upd[j]) continue;
            if (mixed) ++reliable[j];
            const double prev = rmax2[j];
            rmax2[j] = hr[j];
            if (hr[j] <= tol_s[j] * tol_s[j] * bnorm2[j] || it >= maxiter) {
                pending[j] = 1;
                B.h_active[j] = 0;
            } else if (!mixed || hr[j] > 0.25 * prev) {
                B.h_restart[j] = 1;
            }
        }
        if (int rc = sync_flags()) return rc;
    }

    if (B.normal) {
        if (int rc = force_pass(B, *fo)) return rc;
    }
    // solutions: psi_e = I^-1 (eta_e - D_eo psi_o) (the adjoint system: its own
    // blocks), psi_o = x_hi (right form: I^-1 x_hi)
    if (!B.normal) CK(B.psi_odd());
    for (const Group &g : B.groups) {
        if (B.normal) break;
        const Field po = B.psi_o();
        CK(B.hop_group(g, MOBIUS_F64, B.adj() ? 1 : 0, EPI_PRESUB | EPI_M5INV, 0, po, F_PE, F_ETA_E, F_NONE,
                       false));
        CK(launch_unpack_spinor(g.ctx->g, MOBIUS_F64, g.f[F_PE], g.f[po], g.sol, g.nrhs, st));
        B.abytes += 2.0 * g.ctx->g.N5 * 12 * 16 * g.nrhs + 2.0 * g.fb[F_XH] * g.nrhs;
    }
    CK(hipEventRecord(own.ev1, st));
    CK(hipEventSynchronize(own.ev1));
    float ms = 0;
    CK(hipEventElapsedTime(&ms, own.ev0, own.ev1));
    CK(hipEventRecord(own.ev_in, st));
    CK(hipStreamWaitEvent(user, own.ev_in, 0));
    std::vector<double> kap;
    if (int rc = B.kappa(kap)) return rc;
    int status = MOBIUS_OK;
    for (int j = 0; j < nsys; ++j) {
        mobius_solve_info &inf = info[j];
        std::memset(&inf, 0, sizeof(inf));
        inf.iters = iters[j];
        inf.dirac_apps = B.normal ? 4 * iters[j] + 4 * reliable[j] + (fo->grad_links ? 3 : 0)
                                  : 1 + 4 * iters[j] + 2 * reliable[j] + 4;
        inf.reliable_updates = reliable[j];
        inf.status = converged[j] ? MOBIUS_OK : MOBIUS_NOT_CONVERGED;
        inf.true_resid = true_res[j];
        inf.schur_resid = schur_res[j];
        inf.kappa = kap[j];
        inf.err_bound = (B.normal ? kap[j] * kap[j] : kap[j]) * schur_res[j];
        inf.seconds = ms * 1e-3;
        inf.algo_bytes = B.abytes;
        inf.flops = B.aflops;
        if (!converged[j]) status = MOBIUS_NOT_CONVERGED;
    }
    return status;
}

}  // namespace

int batch_solve(mobius_ctx *const *ctxs, int ngroups, const void *const *src, void *const *sol,
                const mobius_solve_opts &o, mobius_solve_info *info, hipStream_t user, bool adjoint)
{
    if (!adjoint && (o.form < 0 || o.form > 3))
        return set_error(MOBIUS_EINVAL, "unknown solve form " + std::to_string(o.form));
    if (!adjoint && o.form == 2) {
        for (int j = 0; j < ngroups; ++j) {
            if (ctxs[j]->sdep)
                return set_error(MOBIUS_EINVAL, "solve form 2 (left form of D^) needs constant b5, c5");
            if (!std::isfinite(b_coeffs(ctxs[j]->c, ctxs[j]->g.Ls).inv_den))
                return set_error(MOBIUS_EINVAL, "solve form 2: B = b5 + c5 C5 is singular");
        }
    }
    const int form = adjoint       ? FORM_ADJ
                     : o.form == 1 ? FORM_RIGHT
                     : o.form == 2 ? FORM_LHAT
                     : o.form == 3 ? FORM_PLAIN
                                   : FORM_LEFT;
    return run(ctxs, ngroups, src, sol, o, info, user, nullptr, form);
}

int force(mobius_ctx *ctx, const void *phi, void *grad_links, void *grad_phi, double *action,
          const mobius_solve_opts &o, mobius_solve_info *info, hipStream_t user)
{
    ForceOut fo{grad_links, grad_phi, 0.0};
    mobius_solve_opts o1 = o;
    o1.nrhs = 1;
    void *sol = nullptr;
    const int rc = run(&ctx, 1, &phi, &sol, o1, info, user, &fo, FORM_LEFT);
    if (rc >= 0) *action = fo.action;
    return rc;
}

}  // namespace mobius
