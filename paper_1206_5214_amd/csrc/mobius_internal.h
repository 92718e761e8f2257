// mobius_internal.h -- private declarations shared by the host side of
// libmobius.so (context, solver) and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mobius.h"

namespace mobius {

// ---------------------------------------------------------------------------
// Geometry and packed layouts
//
// A half lattice of parity p holds Vh = V/2 4d sites.  The packed order of
// the sites of one parity is a bricked traversal: the spatial volume is cut
// into bricks of Bx x By x Bz sites, each brick extended over all t forms a
// column, columns are visited in x-fastest order, and inside a column sites
// run x fastest, then y, z, t.  The t neighbour of a site is then one brick
// cross-section away in the traversal instead of a whole t-slice, which keeps
// all eight neighbours of the sites in flight inside one XCD's L2.
// canon_of[p][i] is the canonical 4d index (x fastest, then y, z, t) of packed
// site i of parity p.  5d sites are Ls-inner: site5 = i * Ls + s.
//
// Spinor field of one parity, storage precision P, is a structure of arrays
// of 16-byte chunks over site5:
//   F64: 12 chunks (one complex each)            -> 192 B / site5
//   F32:  6 chunks (two complex each)            ->  96 B / site5
//   F16:  3 chunks (four complex each, binary16) + one FP32 norm per site5
//                                                ->  52 B / site5
// chunk c of site5 k lives at base + (c * N5 + k) * 16; the F16 norms follow
// the chunks at base + CH * N5 * 16.  Component order is spin * 3 + colour.
//
// Links: for output parity p, 8 directions d: d < 4 is U_d(x), d >= 4 is
// U_{d-4}(x - d^) (undaggered; the kernel applies the dagger), x the packed
// site i of parity p.  Layout [p][8][Vh] of link records: 9 complex<prec>
// (element a*3+b), padded to a multiple of 16 bytes (F64 144 B, F32 80 B,
// F16 48 B) so that a lane reads its link with 16-byte loads.
// Neighbour table nbr[p][Vh][8]: packed index (in parity 1-p) of x + d^ for
// d < 4 and of x - (d-4)^ for d >= 4.

struct Geometry {
    int L[4];
    int Ls;
    int64_t V, Vh, N5;
    int brick[3];                // Bx, By, Bz of the site order
    const int32_t *canon_of;     // device [2][Vh]
};

inline int link_record_bytes(int prec)
{
    return prec == MOBIUS_F64 ? 144 : prec == MOBIUS_F32 ? 80 : 48;
}

inline int64_t field_bytes(const Geometry &g, int prec)
{
    switch (prec) {
    case MOBIUS_F64: return g.N5 * 192;
    case MOBIUS_F32: return g.N5 * 96;
    case MOBIUS_F16: return g.N5 * 52;
    }
    return -1;
}

inline int link_elem_bytes(int prec)
{
    return prec == MOBIUS_F64 ? 16 : prec == MOBIUS_F32 ? 8 : 4;
}

// Per-slice coefficients of the general operator (Sec. 2.1): row s of the
// device table holds LS_B5 .. LS_INV_MP.
enum LsCoef { LS_B5 = 0, LS_C5 = 1, LS_MP = 2, LS_MM = 3, LS_INV_MP = 4, LSC = 5 };

// Scalars of the operator, precomputed on the host.
struct OpCoeffs {
    double b5, c5, mf;
    double Mp, Mm;      // M+ = b5 (4 - M5) + 1, M- = c5 (4 - M5) - 1
    double a;           // M- / M+
    double mu;          // mf * a
    double inv_Mp;      // 1 / M+
    double inv_den;     // 1 / (M+ (1 - mu (-a)^(Ls-1)))
    const double *ls;   // device [Ls][LSC] per-slice b5(s), c5(s), M+(s), M-(s), 1/M+(s);
                        // null: the constant coefficients above
};

// Epilogue program of the hop kernel, applied in this order to r = -1/2 H (B in):
enum Epilogue : int {
    EPI_BDAG = 1,      // r = B^+ r          (always set for the adjoint hop)
    EPI_M5ADD = 2,     // r = I y + r        (y: same-parity input; full operator)
    EPI_PRESUB = 4,    // r = x - r
    EPI_M5INV = 8,     // r = I^-1 r  (I^-+ r for the adjoint)
    EPI_POSTSUB = 16,  // r = x - r
    EPI_NORM = 32,     // partial sums of |r|^2 (FP64)
    EPI_BMIX = 64,     // r = B r  (after EPI_M5INV; stores the input of a premixed hop)
    EPI_PREMIXED = 128,  // forward hop whose input already holds B in: r = -1/2 H in
    EPI_NOBOUT = 256,  // adjoint hop without its output B^+: r = -1/2 H^+ in (the left form's
                       // adjoint, whose B^+ acts on the input); EPI_BMIX then applies B^+
    EPI_M5SUB = 512,   // r = I y - r (I^+ y - r in the adjoint hop): the Schur complement itself
};

struct HopArgs {
    int prec;
    int dag;            // 0: D block, 1: D^+ block
    int epi;            // Epilogue bit mask
    int out_parity;
    const void *in;     // parity 1 - out_parity
    void *out;          // parity out_parity
    const void *x;      // same parity as out (PRESUB/POSTSUB), may be null
    const void *y;      // same parity as out (M5ADD), may be null
    double *partials;   // per-block |r|^2 (EPI_NORM), [rhs][pstride]
    int nrhs;
    const int32_t *active = nullptr;  // per-rhs flags in device memory (null: all)
    int64_t fstride = 0;  // bytes between rhs fields (0: one field)
    int64_t pstride = 0;  // partial slots per rhs (0: the number of blocks)
    const struct HopTuning *tune = nullptr;  // launch parameters (null: process defaults)
};

// Kernel arguments of one hop launch over one lattice and nrhs fields (rhs r
// at base + r * fstride); also the descriptor of one group of a batch.
struct HopParams {
    const char *in;
    char *out;
    const char *x;
    const char *y;
    const char *links;      // parity block of the packed links
    const int32_t *nbr;     // parity block of the neighbour table
    double *partials;       // [rhs][pstride], one slot per block
    const int32_t *active;  // per-rhs flag (null: all); a zero skips that rhs
    int64_t Vh, N5;
    int64_t fstride, pstride, nblocks;
    int Ls, spw, nrhs;
    int remap;              // XCD-contiguous block order
    int stage_links;        // copy the block's links to LDS first
    int m5_off;             // byte offset in dynamic LDS of the I^-1 epilogue's buffer: 0 (it
                            // reuses the staged links' space once the direction loop is done)
                            // or past the links (nrhs > 1: the links serve every system)
    int nt;                 // non-temporal loads of the links
    int pf;                 // prefetch depth of the direction loop (0, 1, 2); 3: FP16 matrix-core
                            // colour multiply (requires stage_links and Ls % 4 == 0)
    OpCoeffs c;
};

// Launch parameters of the hop kernel chosen at run time.  The process
// defaults are the values measured best at 24^3x64, Ls=12 (environment
// overrides: MOBIUS_XCD_REMAP=0/1 block order, MOBIUS_PREFETCH=0/1/2 software
// pipelining depth of the direction loop, MOBIUS_STAGE_LINKS=0/1,
// MOBIUS_NT_LINKS=0/1); every context holds its own copy per precision, which
// mobius_tune replaces by the fastest measured candidate.
struct HopTuning {
    int xcd_remap = 1;
    int prefetch = -1;     // 0, 1 (next neighbour spinor), 2 (and its link); -1: per precision
    int stage_links = 1;   // copy each block's links to LDS once
    int nt_links = 0;      // non-temporal link loads
    int mfma = 1;          // FP16: colour multiply on the matrix cores where the lane map allows
};
// prefetch depth used for a precision (measured at 24^3x64, Ls=12: the FP64
// hop needs more than 256 VGPRs once a neighbour is prefetched, which halves
// its occupancy -- 967 us at depth 0 against 1262 us at depth 1; FP32 and FP16
// gain a few percent from depth 2)
inline int prefetch_depth(const HopTuning &t, int prec)
{
    if (t.prefetch >= 0) return t.prefetch;
    return prec == MOBIUS_F64 ? 0 : 2;
}
// Brick of the site order for a lattice: MOBIUS_BRICK="bx,by,bz" overrides.
void choose_brick(const int L[4], int Ls, int brick[3]);
HopTuning &hop_tuning();

// Reduction workspace sizing: number of blocks a site kernel launches.
int64_t site_kernel_blocks(const Geometry &g);

// ---------------------------------------------------------------------------
// Kernel launchers (mobius_kernels.hip)

// nbr from canon_of and its inverse packed_of[V] (index of a canonical site
// inside its parity)
hipError_t launch_build_geometry(const Geometry &g, const int32_t *packed_of, int32_t *nbr,
                                 hipStream_t st);
hipError_t launch_pack_links(const Geometry &g, int prec, const void *canon, void *packed,
                             hipStream_t st,
                             double sf = 1.0, double sb = 1.0);
// F = TA(U G^+) per link (canonical complex128 3x3 records, nlinks of them)
hipError_t launch_lie_force(int64_t nlinks, const void *U, const void *G, void *F, hipStream_t st);
// 4d field on the walls of the fifth dimension and back (canonical layouts)
hipError_t launch_wall_place(const Geometry &g, const void *b4, void *eta5, int nrhs, hipStream_t st);
hipError_t launch_wall_read(const Geometry &g, const void *psi5, void *q4, int nrhs, hipStream_t st);
// bulk reconstruction: Psi_0 = psi4, Psi_s = -(P- y_s + P+ y_{s-1}) for s > 0 (canonical layouts)
hipError_t launch_bulk_assemble(const Geometry &g, const void *psi4, const void *y5, void *Psi5,
                                int nrhs, hipStream_t st);
hipError_t launch_pack_spinor(const Geometry &g, int prec, const void *canon, void *even, void *odd,
                              int nrhs, hipStream_t st);
hipError_t launch_unpack_spinor(const Geometry &g, int prec, const void *even, const void *odd,
                                void *canon, int nrhs, hipStream_t st);
hipError_t launch_hop(const Geometry &g, const OpCoeffs &c, const void *links, const int32_t *nbr,
                      const HopArgs &a, hipStream_t st);
HopParams make_hop_params(const Geometry &g, const OpCoeffs &c, const void *links,
                          const int32_t *nbr, const HopArgs &a);
size_t hop_link_lds_bytes(int prec, int Ls, bool rows);
// bytes of the I^-1 epilogue's LDS buffer (one block) for a storage precision
size_t m5_epilogue_lds_bytes(int prec);
// persistent launch over groups (device array) with block prefix sums prefix[0..n]
hipError_t launch_hop_batch(int prec, int dag, int epi, const HopParams *groups_dev, int ngroups,
                            const int64_t *prefix_dev, size_t lds_bytes, int grid, int pf,
                            hipStream_t st);
// Per-site s-direction operators on one packed half field:
//   kind 0: out = I in (dag: I^+ in); kind 1: out = I^-1 in (dag: I^-+ in)
hipError_t launch_m5(const Geometry &g, const OpCoeffs &c, int prec, int kind, int dag,
                     const void *in, void *out, int nrhs, hipStream_t st);

// BLAS-1 on packed half fields (storage precision prec), FP64 scalars in
// device memory, FP64 partial sums per block (deterministic fixed-order
// reduction in launch_reduce_batch).
int64_t blas_blocks(const Geometry &g);
// Allocation-free workspace: a static device array of NOALLOC_SCRATCH_BYTES
// per GPU.  noalloc_scratch_init (with `device` current) looks up its address
// on that device once; noalloc_scratch returns it (null before init).
constexpr int64_t NOALLOC_SCRATCH_BYTES = (int64_t)64 << 20;
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
// fill with zeros (kernel, not hipMemset, so it is safe under graph capture)
hipError_t launch_zero(void *ptr, int64_t bytes, hipStream_t st);
// a packed field of n5 5d sites with seeded values of Gaussian-field magnitude
hipError_t launch_fill_random(int prec, void *ptr, int64_t n5, uint32_t seed, hipStream_t st);
// Scalar updates of CGLS, on device (one thread per system):
// Most search directions one chunk of a mixed-precision CGLS keeps for its
// deferred x update.
constexpr int RING_MAX = 16;

struct CgScalars {
    double gamma;      // |s|^2 of the current direction
    double qq;         // |q|^2
    double rr;         // |r|^2
    double gamma_new;
    double alpha, beta;
    // Coefficient history for the Lanczos estimate of the condition number:
    // hist[k] = (beta_{k-1}, alpha_k) of iteration k (beta_{k-1} = 0 at the
    // first step of a Krylov segment), kept for the first hmax iterations.
    double *hist;
    int64_t nhist, hmax;
    // alpha of each iteration of a chunk whose x update is deferred to the
    // chunk's end (slot = the iteration's index in the chunk)
    double aring[RING_MAX];
};

// One system (one lattice, one right-hand side) of a batched vector kernel.
// Field roles per kernel:
//   VEC_CG_XR       a = x (prec2; null: no x update), b = p, c = r, d = q, s0 = alpha; |r|^2 partials
//   VEC_AXPBY(_NORM) d = s0 a + s1 b (null scalar = 1) [; |d|^2 partials]
//   VEC_NORM2       |a|^2 partials
//   VEC_CONVERT     b (prec2) = a (prec)
//   VEC_ACCUMULATE  d (FP64) += a (prec); a = 0
//   VEC_DOT         Re <a, b> partials (a and b in precision prec)
//   VEC_PUPD_X      c (prec2) += s0 b;  b = a + s1 b          (x += alpha p_old; p = s + beta p_old)
//   VEC_XFLUSH      c (prec2) += s0 a                          (x += alpha p)
//   VEC_PUPD_RING   p[slot] = a + s1 p[prev]                   (b = p[0]; slots sstride bytes apart)
//   VEC_XRING       c (prec2) += sum_{i < n} s0[i] p[i]        (b = p[0]; slots sstride bytes apart)
struct VecSys {
    char *a, *b, *c, *d;
    const double *s0, *s1;
    int64_t sstride;       // bytes between the slots of a ring of directions
    double *partials;      // this system's partial slots
    int64_t nparts;        // number of valid partial slots (for the reduction)
    int64_t N5;
    int32_t flag;          // index into the active flags (-1: always active)
    int32_t Ls;            // fifth-dimension extent of the system's lattice
    const OpCoeffs *coef;  // operator coefficients of the system's lattice (device)
};
enum VecKind { VEC_CG_XR, VEC_AXPBY, VEC_AXPBY_NORM, VEC_NORM2, VEC_CONVERT, VEC_ACCUMULATE,
               VEC_DOT, VEC_PUPD_X, VEC_XFLUSH, VEC_PUPD_RING, VEC_XRING };
hipError_t launch_vec_batch(int kind, int prec, int prec2, const VecSys *sys_dev, int nsys,
                            int64_t max_n5, const int32_t *active, hipStream_t st);
// out[sys * out_stride] = sum of partials[0 .. count) of each system (count_override > 0)
// or of its own nparts
hipError_t launch_reduce_batch(const VecSys *sys_dev, int nsys, const int32_t *active,
                               int64_t count_override, double *out, int64_t out_stride,
                               hipStream_t st);
// VEC_PUPD_RING (a0 = slot, a1 = prev) or VEC_XRING (a0 = n) over a ring of
// directions; prec: the directions, prec2: x
hipError_t launch_ring_batch(int kind, int prec, int prec2, const VecSys *sys_dev, int nsys,
                             int64_t max_n5, const int32_t *active, int a0, int a1, hipStream_t st);
// op 0: alpha = gamma / qq (also kept in aring[slot] when slot >= 0);
// op 1: beta, gamma;  op 2: alpha = 0
hipError_t launch_cg_scalar_batch(CgScalars *sc, int nsys, int op, const int32_t *active,
                                  int32_t *restart, hipStream_t st, int slot = -1);
// r = a -= s0 b (|r|^2 partials per site block) and c = I^-+ r (mode 0), c =
// I^-1 r (mode 1), nothing (mode 2) or c = B^+ I^-+ r (mode 3, constant
// coefficients), in the site-lane mapping of the hop
// (one workgroup per site block and system); max_blocks is the largest number
// of site blocks of any system
hipError_t launch_rupd_m5inv_batch(int prec, const VecSys *sys_dev, int nsys, int64_t max_blocks,
                                   const int32_t *active, int mode, hipStream_t st);

// Link derivative of the pseudofermion action (mobius_force.hip): for the
// sites y of one parity p, grad[mu][canon(y)] (complex128 3x3, canonical link
// layout) from FP64 packed fields L_p, R_p (parity p) and L_{1-p}, R_{1-p}.
struct ForceParams {
    const char *Lp, *Rp, *Ln, *Rn;
    const int32_t *nbr;       // parity block of the neighbour table
    const int32_t *canon_of;  // parity block of the site order
    double2 *grad;
    int64_t Vh, N5, V;
    int Ls, spw;
    double scale;     // grad = scale * G (accumulate: grad += scale * G)
    int accumulate;
    double ef, eb;    // e^{+mu}, e^{-mu}: the chemical potential's factors of the
                      // forward and backward time-like hop of D_DW
    OpCoeffs c;
};
// G of 2 Re <L, dD_hop R> (D_hop = -1/2 H B, the hopping part of D_DW with the
// coefficients c) for the links U_mu(y) of the sites y of parity `parity`
hipError_t launch_force(const Geometry &g, const OpCoeffs &c, int parity, const int32_t *nbr,
                        const void *Lp, const void *Rp, const void *Ln, const void *Rn,
                        void *grad, hipStream_t st, double scale = 1.0, bool accumulate = false,
                        double mu = 0.0);
// *out = sum of |x_k|^2 over n doubles (FP64 partial sums per block in
// partials[nblocks], fixed-order reduction); nblocks = norm2_blocks(n)
int64_t norm2_blocks(int64_t n);
hipError_t launch_norm2_f64(const double *x, int64_t n, double *partials, double *out, hipStream_t st);

// device buffer owned by a context
struct DevBuf {
    void *p = nullptr;
    int64_t bytes = 0;
    hipError_t ensure(int64_t b)
    {
        if (b <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// error reporting shared by the host files (message readable through mobius_last_error)
int set_error(int code, const std::string &msg);

// Forms of the Schur system the CG iterates on (Sec. 3): the left-preconditioned
// D_pre, the right-preconditioned D_R = I D_pre I^-1 (on z = I psi_o), and the
// left form of the adjoint matrix D_DW^+ (for D_DW^+ psi = eta).
// FORM_LHAT iterates on the Schur operator of the left form D^ = D-^-1 D_DW D-
// of Sec. 2.1, 1 - I^-1 D^_oe I^-1 D^_eo = B D_pre B^-1 (constant coefficients),
// on y = B psi_o: every hop of its CG step applies B after the hopping sum, so
// none gathers the s-neighbours of its input.
// FORM_PLAIN iterates on the Schur complement itself, S = I - D_oe I^-1 D_eo
// (D_pre = I^-1 S), on psi_o.
enum SchurForm { FORM_LEFT = 0, FORM_RIGHT = 1, FORM_LHAT = 2, FORM_ADJ = 3, FORM_PLAIN = 4 };
// coefficients of I with (M+, M-) replaced by (b5, c5): the same elimination
// then applies B = b5 + c5 C5 (kind 0) or B^-1 (kind 1) through launch_m5
OpCoeffs b_coeffs(const OpCoeffs &c, int Ls);

// Batched red/black CG: ngroups lattices (contexts), each with nrhs systems;
// opts.form selects left or right preconditioning; adjoint solves D_DW^+ psi = eta.
int batch_solve(mobius_ctx *const *ctxs, int ngroups, const void *const *src, void *const *sol,
                const mobius_solve_opts &opts, mobius_solve_info *info, hipStream_t stream,
                bool adjoint = false);
// Time the hop launch candidates for one precision; keep the best in ctx.
int tune(mobius_ctx *ctx, int prec, int reps, mobius_tune_result *out, hipStream_t st);

// S = phi_o^+ (D_pre^+ D_pre)^-1 phi_o with its link and source gradients.
int force(mobius_ctx *ctx, const void *phi, void *grad_links, void *grad_phi, double *action,
          const mobius_solve_opts &opts, mobius_solve_info *info, hipStream_t stream);

}  // namespace mobius

struct mobius_ctx {
    mobius_params P{};
    mobius::Geometry g{};
    mobius::OpCoeffs c{};
    int device = 0;
    mobius::DevBuf canon_of;  // [2][Vh] canonical index of each packed site
    mobius::DevBuf nbr;
    mobius::DevBuf links[3];
    mobius::DevBuf links_dag[3];  // adjoint's records when a chemical potential is set
    bool has_mu = false;
    mobius::DevBuf scratch;   // operator temporaries (SCHUR blocks)
    mobius::DevBuf work;      // solver fields
    mobius::DevBuf partials;  // reduction partials
    mobius::DevBuf scalars;   // solver scalars, flags and descriptor tables
    mobius::DevBuf prop;      // 4d propagator temporaries (canonical and packed 5d fields)
    mobius::DevBuf ls_coef;   // per-slice coefficient table [Ls][LSC] (s-dependent b5, c5)
    bool sdep = false;        // the operator has per-slice coefficients
    hipStream_t solve_stream = nullptr;
    mobius::HopTuning tune[3];  // hop launch parameters per storage precision
    double tuned_us[3] = {0, 0, 0};  // hop time of the tuned parameters (0: not tuned)
    // Pauli-Villars view (mf = 1) of the same lattice for the solves of the
    // bulk reconstruction: shares (borrows) the site tables, links and
    // coefficient table of its parent, owns its solver buffers
    mobius_ctx *pv = nullptr;
    bool borrowed = false;
};

// Link records a hop reads: with a chemical potential the adjoint hops use
// their own records (factors e^{-+mu} instead of e^{+-mu} on the time-like ones).
inline const void *hop_links(const mobius_ctx *ctx, int prec, int dag)
{
    return (dag && ctx->has_mu) ? ctx->links_dag[prec].p : ctx->links[prec].p;
}
