// mobius_api.cpp -- C ABI of libmobius.so: context, red/black operator blocks
// and the CGLS solvers (plain FP64, and low-precision operator with FP64
// reductions, reliable updates and outer defect correction).
#include "mobius_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace mobius;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

}  // namespace

int mobius::set_error(int code, const std::string &msg) { return fail(code, msg); }

namespace {

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MOBIUS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

}  // namespace

namespace {

OpCoeffs make_coeffs(const mobius_params &p)
{
    OpCoeffs c{};
    c.b5 = p.b5;
    c.c5 = p.c5;
    c.mf = p.mf;
    c.Mp = p.b5 * (4.0 - p.M5) + 1.0;
    c.Mm = p.c5 * (4.0 - p.M5) - 1.0;
    c.a = c.Mm / c.Mp;
    c.mu = p.mf * c.a;
    c.inv_Mp = 1.0 / c.Mp;
    c.inv_den = 1.0 / (c.Mp * (1.0 - c.mu * std::pow(-c.a, p.Ls - 1)));
    c.ls = nullptr;
    return c;
}

}  // namespace

OpCoeffs mobius::b_coeffs(const OpCoeffs &c, int Ls)
{
    // B = b5 + c5 C5 has the shape of I = M+ + M- C5 (Sec. 3), so the same
    // closed-form elimination inverts it with (M+, M-) -> (b5, c5)
    OpCoeffs b = c;
    b.Mp = c.b5;
    b.Mm = c.c5;
    b.a = c.c5 / c.b5;
    b.mu = c.mf * b.a;
    b.inv_Mp = 1.0 / c.b5;
    b.inv_den = 1.0 / (c.b5 * (1.0 - b.mu * std::pow(-b.a, Ls - 1)));
    b.ls = nullptr;
    return b;
}

namespace {

// Per-slice table of the general operator (Sec. 2.1) from the caller's
// b5(s), c5(s); false if the Ls-direction block is singular: some M+(s) = 0,
// or a vanishing pivot d + k g of the cyclic elimination of either chirality
// (the product g of the row ratios -M-(t)/M+(t) over the Ls-1 rows, the same
// for I and its transpose), for the quark mass and for the Pauli-Villars mass 1.
bool ls_table(const mobius_params &p, std::vector<double> &tab)
{
    const int Ls = p.Ls;
    tab.assign((size_t)Ls * LSC, 0.0);
    for (int s = 0; s < Ls; ++s) {
        const double b = p.b5s ? p.b5s[s] : p.b5, c = p.c5s ? p.c5s[s] : p.c5;
        const double Mp = b * (4.0 - p.M5) + 1.0, Mm = c * (4.0 - p.M5) - 1.0;
        if (!std::isfinite(b) || !std::isfinite(c) || Mp == 0.0) return false;
        double *r = &tab[(size_t)s * LSC];
        r[LS_B5] = b;
        r[LS_C5] = c;
        r[LS_MP] = Mp;
        r[LS_MM] = Mm;
        r[LS_INV_MP] = 1.0 / Mp;
    }
    for (double mf : {p.mf, 1.0}) {
        double gu = 1.0, gl = 1.0;  // upper form: rows 0..Ls-2; lower form: rows Ls-1..1
        for (int t = 0; t < Ls - 1; ++t) gu *= -tab[t * LSC + LS_MM] / tab[t * LSC + LS_MP];
        for (int t = Ls - 1; t > 0; --t) gl *= -tab[t * LSC + LS_MM] / tab[t * LSC + LS_MP];
        const double km = -mf * tab[(Ls - 1) * LSC + LS_MM], kp = -mf * tab[LS_MM];
        const double pu = tab[(Ls - 1) * LSC + LS_MP] + km * gu;  // P- of I
        const double pl = tab[LS_MP] + kp * gl;                   // P+ of I
        if (!(std::isfinite(pu) && std::isfinite(pl)) || pu == 0.0 || pl == 0.0) return false;
    }
    return true;
}

int check_ctx(const mobius_ctx *ctx)
{
    if (!ctx) return fail(MOBIUS_EINVAL, "null context");
    return MOBIUS_OK;
}

int check_prec(int prec)
{
    if (prec != MOBIUS_F64 && prec != MOBIUS_F32 && prec != MOBIUS_F16)
        return fail(MOBIUS_EINVAL, "unknown precision " + std::to_string(prec));
    return MOBIUS_OK;
}

hipStream_t S(void *stream) { return static_cast<hipStream_t>(stream); }

// Bricked site order (see mobius_internal.h): columns of bx x by x bz sites
// over all t, columns x fastest, inside a column x, y, z, then t.
void site_order(const Geometry &g, std::vector<int32_t> &canon_of, std::vector<int32_t> &packed_of)
{
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int bx = g.brick[0], by = g.brick[1], bz = g.brick[2];
    canon_of.assign(2 * g.Vh, -1);
    packed_of.assign(g.V, -1);
    int64_t n[2] = {0, 0};
    for (int z0 = 0; z0 < Lz; z0 += bz)
        for (int y0 = 0; y0 < Ly; y0 += by)
            for (int x0 = 0; x0 < Lx; x0 += bx)
                for (int t = 0; t < Lt; ++t)
                    for (int z = z0; z < std::min(z0 + bz, Lz); ++z)
                        for (int y = y0; y < std::min(y0 + by, Ly); ++y)
                            for (int x = x0; x < std::min(x0 + bx, Lx); ++x) {
                                const int64_t c = ((int64_t)(t * Lz + z) * Ly + y) * Lx + x;
                                const int p = (x + y + z + t) & 1;
                                packed_of[c] = (int32_t)n[p];
                                canon_of[p * g.Vh + n[p]] = (int32_t)c;
                                ++n[p];
                            }
}

}  // namespace

namespace mobius {

// Site-order brick: among bricks whose sides divide the lattice (bx even),
// the largest whose one-site-thick slice of an FP64 field (bx by bz / 2 sites
// x Ls x 192 B) stays within 2 MiB, half of one XCD's L2, so that the t
// neighbours one slice away are still cached; ties go to the smaller surface.
// (At 24^3 x 64, Ls = 12 this is 12^3, one column per XCD, which measured
// fastest among bricks from 2^3 to 24^3.)
void choose_brick(const int L[4], int Ls, int brick[3])
{
    if (const char *e = std::getenv("MOBIUS_BRICK")) {
        int b[3];
        if (std::sscanf(e, "%d,%d,%d", &b[0], &b[1], &b[2]) == 3 && b[0] > 0 && b[1] > 0 && b[2] > 0) {
            for (int k = 0; k < 3; ++k) brick[k] = std::min(b[k], L[k]);
            return;
        }
    }
    const double budget = 2.0 * 1024.0 * 1024.0;
    const double per_site = 0.5 * Ls * 192.0;
    brick[0] = 2;
    brick[1] = brick[2] = 1;
    double best_vol = 0, best_surf = 1e30;
    for (int bx = 2; bx <= L[0]; bx += 2) {
        if (L[0] % bx) continue;
        for (int by = 1; by <= L[1]; ++by) {
            if (L[1] % by) continue;
            for (int bz = 1; bz <= L[2]; ++bz) {
                if (L[2] % bz) continue;
                const double vol = (double)bx * by * bz;
                if (vol * per_site > budget) continue;
                const double surf = 1.0 / bx + 1.0 / by + 1.0 / bz;
                if (vol > best_vol || (vol == best_vol && surf < best_surf)) {
                    best_vol = vol;
                    best_surf = surf;
                    brick[0] = bx;
                    brick[1] = by;
                    brick[2] = bz;
                }
            }
        }
    }
}

}  // namespace mobius

// ---------------------------------------------------------------------------

extern "C" const char *mobius_last_error(void) { return g_err.c_str(); }

extern "C" int mobius_create(mobius_ctx **out, const mobius_params *p, const void *links_c128,
                             void *stream)
{
    g_err.clear();
    if (!out || !p || !links_c128) return fail(MOBIUS_EINVAL, "null argument to mobius_create");
    *out = nullptr;
    for (int mu = 0; mu < 4; ++mu)
        if (p->L[mu] < 2 || (p->L[mu] & 1))
            return fail(MOBIUS_EINVAL, "every lattice extent must be even and >= 2");
    if (p->Ls < 2 || p->Ls > 64) return fail(MOBIUS_EINVAL, "Ls must be in [2, 64]");
    const bool sdep = p->b5s || p->c5s;
    std::vector<double> tab;
    if (sdep) {
        if (!ls_table(*p, tab)) return fail(MOBIUS_EINVAL, "the Ls-direction block I is singular "
                                                           "or a per-slice coefficient is not finite");
    } else {
        const double Mp = p->b5 * (4.0 - p->M5) + 1.0;
        if (Mp == 0.0) return fail(MOBIUS_EINVAL, "M+ = b5 (4 - M5) + 1 is zero");
    }
    OpCoeffs c = make_coeffs(*p);
    if (!sdep && !std::isfinite(c.inv_den)) return fail(MOBIUS_EINVAL, "the Ls-direction block I is singular");
    if (!std::isfinite(p->mu) || std::fabs(p->mu) > 10.0)
        return fail(MOBIUS_EINVAL, "the chemical potential must be finite with |mu| <= 10");
    const bool own_brick = p->brick[0] || p->brick[1] || p->brick[2];
    for (int k = 0; k < 3 && own_brick; ++k)
        if (p->brick[k] < 1 || p->brick[k] > p->L[k])
            return fail(MOBIUS_EINVAL, "each side of the site-order brick must lie in 1..L");

    mobius_ctx *ctx = new mobius_ctx();
    ctx->P = *p;
    ctx->P.b5s = ctx->P.c5s = nullptr;  // the caller's arrays are not kept
    ctx->sdep = sdep;
    ctx->c = c;
    ctx->has_mu = p->mu != 0.0;
    Geometry &g = ctx->g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = p->L[mu];
    g.Ls = p->Ls;
    g.V = (int64_t)p->L[0] * p->L[1] * p->L[2] * p->L[3];
    g.Vh = g.V / 2;
    g.N5 = g.Vh * g.Ls;
    // every packed array is addressed through one buffer descriptor with a
    // 32-bit range: the largest (an FP64 field, one parity of FP64 links) must fit
    if (field_bytes(g, MOBIUS_F64) > (int64_t)UINT32_MAX ||
        (int64_t)8 * g.Vh * link_record_bytes(MOBIUS_F64) > (int64_t)UINT32_MAX) {
        delete ctx;
        return fail(MOBIUS_EINVAL, "lattice too large: an FP64 half field must stay below 4 GiB");
    }
    hipStream_t st = S(stream);
    auto cleanup = [&](int code) {
        mobius_destroy(ctx);
        return code;
    };
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
    // address of this device's workspace of mobius_dslash_noalloc (set up
    // here, with the device current, so that the entry point allocates nothing)
    e = noalloc_scratch_init(ctx->device);
    if (e != hipSuccess)
        return cleanup(fail(MOBIUS_EHIP, std::string("workspace address: ") + hipGetErrorString(e)));
    if (sdep) {
        e = ctx->ls_coef.ensure((int64_t)(tab.size() * sizeof(double)));
        if (e == hipSuccess)
            e = hipMemcpy(ctx->ls_coef.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
        ctx->c.ls = static_cast<const double *>(ctx->ls_coef.p);
    }
    // site order and neighbour table
    choose_brick(g.L, g.Ls, g.brick);
    if (own_brick)
        for (int k = 0; k < 3; ++k) g.brick[k] = p->brick[k];
    std::vector<int32_t> canon_of, packed_of;
    site_order(g, canon_of, packed_of);
    DevBuf packed_dev;
    e = ctx->canon_of.ensure(2 * g.Vh * (int64_t)sizeof(int32_t));
    if (e == hipSuccess) e = packed_dev.ensure(g.V * (int64_t)sizeof(int32_t));
    if (e == hipSuccess) e = ctx->nbr.ensure(2 * 8 * g.Vh * (int64_t)sizeof(int32_t));
    if (e != hipSuccess) {
        packed_dev.release();
        return cleanup(fail(MOBIUS_ENOMEM, "site tables: " + std::string(hipGetErrorString(e))));
    }
    g.canon_of = static_cast<const int32_t *>(ctx->canon_of.p);
    e = hipMemcpy(ctx->canon_of.p, canon_of.data(), canon_of.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(packed_dev.p, packed_of.data(), packed_of.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_build_geometry(g, static_cast<const int32_t *>(packed_dev.p), static_cast<int32_t *>(ctx->nbr.p), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    packed_dev.release();
    if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
    for (int prec = 0; prec < 3; ++prec) {
        ctx->tune[prec] = hop_tuning();
        ctx->tune[prec].prefetch = prefetch_depth(hop_tuning(), prec);
        // a chemical potential enters the time-like records: e^{+mu} forward,
        // e^{-mu} backward, and the opposite in the adjoint's own records
        const double ef = std::exp(p->mu), eb = std::exp(-p->mu);
        e = ctx->links[prec].ensure(2 * 8 * g.Vh * (int64_t)link_record_bytes(prec));
        if (e != hipSuccess) return cleanup(fail(MOBIUS_ENOMEM, "links: " + std::string(hipGetErrorString(e))));
        e = launch_pack_links(g, prec, links_c128, ctx->links[prec].p, st, ef, eb);
        if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
        if (ctx->has_mu) {
            e = ctx->links_dag[prec].ensure(2 * 8 * g.Vh * (int64_t)link_record_bytes(prec));
            if (e != hipSuccess)
                return cleanup(fail(MOBIUS_ENOMEM, "links: " + std::string(hipGetErrorString(e))));
            e = launch_pack_links(g, prec, links_c128, ctx->links_dag[prec].p, st, eb, ef);
            if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
        }
    }
    *out = ctx;
    return MOBIUS_OK;
}

extern "C" int mobius_destroy(mobius_ctx *ctx)
{
    if (!ctx) return MOBIUS_OK;
    (void)hipDeviceSynchronize();
    if (ctx->pv) mobius_destroy(ctx->pv);
    if (!ctx->borrowed) {
        ctx->nbr.release();
        ctx->canon_of.release();
        for (auto &l : ctx->links) l.release();
        for (auto &l : ctx->links_dag) l.release();
        ctx->ls_coef.release();
    }
    ctx->scratch.release();
    ctx->work.release();
    ctx->partials.release();
    ctx->scalars.release();
    ctx->prop.release();
    if (ctx->solve_stream) (void)hipStreamDestroy(ctx->solve_stream);
    delete ctx;
    return MOBIUS_OK;
}

extern "C" int64_t mobius_field_bytes(const mobius_ctx *ctx, int32_t prec)
{
    if (!ctx || check_prec(prec) != MOBIUS_OK) return -1;
    return field_bytes(ctx->g, prec);
}

extern "C" int mobius_pack(mobius_ctx *ctx, int32_t prec, const void *canon, void *even, void *odd,
                           int32_t nrhs, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_prec(prec)) return r;
    if (!canon || !even || !odd || nrhs < 1) return fail(MOBIUS_EINVAL, "bad argument to mobius_pack");
    if (even == odd) return fail(MOBIUS_EINVAL, "even and odd outputs alias");
    HIPCHK(launch_pack_spinor(ctx->g, prec, canon, even, odd, nrhs, S(stream)));
    return MOBIUS_OK;
}

extern "C" int mobius_unpack(mobius_ctx *ctx, int32_t prec, const void *even, const void *odd,
                             void *canon, int32_t nrhs, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_prec(prec)) return r;
    if (!canon || !even || !odd || nrhs < 1) return fail(MOBIUS_EINVAL, "bad argument to mobius_unpack");
    HIPCHK(launch_unpack_spinor(ctx->g, prec, even, odd, canon, nrhs, S(stream)));
    return MOBIUS_OK;
}

namespace {

HopArgs hop_args(int prec, int dag, int epi, int out_parity, const void *in, void *out,
                 const void *x = nullptr, const void *y = nullptr, double *partials = nullptr,
                 int nrhs = 1)
{
    HopArgs a;
    a.prec = prec;
    a.dag = dag;
    a.epi = epi;
    a.out_parity = out_parity;
    a.in = in;
    a.out = out;
    a.x = x;
    a.y = y;
    a.partials = partials;
    a.nrhs = nrhs;
    return a;
}

hipError_t hop(mobius_ctx *ctx, const HopArgs &a0, hipStream_t st)
{
    HopArgs a = a0;
    a.tune = &ctx->tune[a.prec];
    return launch_hop(ctx->g, ctx->c, hop_links(ctx, a.prec, a.dag), static_cast<const int32_t *>(ctx->nbr.p),
                      a, st);
}

// D_pre (dag = 0) or D_pre^+ (dag = 1) on odd fields; t_even and u_odd are
// temporaries of the same precision.  Optional partials receive |out|^2.
hipError_t schur(mobius_ctx *ctx, int prec, int dag, const void *in, void *out, void *t_even,
                 void *u_odd, double *partials, int nrhs, hipStream_t st)
{
    hipError_t e;
    const int norm = partials ? EPI_NORM : 0;
    if (!dag) {
        // t = B I^-1 D_eo in ;  out = in - I^-1 D_oe (t already mixed in s)
        e = hop(ctx, hop_args(prec, 0, EPI_M5INV | EPI_BMIX, 0, in, t_even, nullptr, nullptr, nullptr, nrhs),
                st);
        if (e != hipSuccess) return e;
        return hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB | norm, 1, t_even, out,
                                 in, nullptr, partials, nrhs), st);
    }
    // u = I^-+ in ;  t = I^-+ (D_oe)^+ u ;  out = in - (D_eo)^+ t
    e = launch_m5(ctx->g, ctx->c, prec, 1, 1, in, u_odd, nrhs, st);
    if (e != hipSuccess) return e;
    e = hop(ctx, hop_args(prec, 1, EPI_M5INV, 0, u_odd, t_even, nullptr, nullptr, nullptr, nrhs), st);
    if (e != hipSuccess) return e;
    return hop(ctx, hop_args(prec, 1, EPI_POSTSUB | norm, 1, t_even, out, in, nullptr, partials, nrhs),
               st);
}

// fixed_scratch: caller-provided workspace of fixed_bytes for the SCHUR
// temporaries (null: the context's own, allocated on first use)
int dslash_common(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity, const void *in,
                  void *out, int32_t nrhs, void *stream, int dag, void *fixed_scratch = nullptr,
                  int64_t fixed_bytes = 0)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_prec(prec)) return r;
    if (!in || !out || nrhs < 1) return fail(MOBIUS_EINVAL, "null field or nrhs < 1");
    if (in == out) return fail(MOBIUS_EINVAL, "in and out alias");
    if (out_parity != 0 && out_parity != 1) return fail(MOBIUS_EINVAL, "out_parity must be 0 or 1");
    hipStream_t st = S(stream);
    switch (op) {
    case MOBIUS_OP_HOP:
        HIPCHK(hop(ctx, hop_args(prec, dag, 0, out_parity, in, out, nullptr, nullptr, nullptr, nrhs), st));
        return MOBIUS_OK;
    case MOBIUS_OP_M5:
        HIPCHK(launch_m5(ctx->g, ctx->c, prec, 0, dag, in, out, nrhs, st));
        return MOBIUS_OK;
    case MOBIUS_OP_FULL: {
        // in, out: the nrhs even fields followed by the nrhs odd fields;
        // out_p = D_{p,1-p} in_{1-p} + I in_p (daggered blocks for the adjoint)
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        const char *ie = static_cast<const char *>(in), *io = ie + fb;
        char *oe = static_cast<char *>(out), *oo = oe + fb;
        if (oe < io + fb && ie < oo + fb) return fail(MOBIUS_EINVAL, "in and out overlap");
        HIPCHK(hop(ctx, hop_args(prec, dag, EPI_M5ADD, 0, io, oe, nullptr, ie, nullptr, nrhs), st));
        HIPCHK(hop(ctx, hop_args(prec, dag, EPI_M5ADD, 1, ie, oo, nullptr, io, nullptr, nrhs), st));
        return MOBIUS_OK;
    }
    case MOBIUS_OP_SCHUR_RIGHT: {
        // D_R = 1 - D_oe I^-1 D_eo I^-1 (v = I^-1 in, t = B I^-1 D_eo v, out = in - D_oe t);
        // D_R^+ = 1 - I^-+ D_eo^+ I^-+ D_oe^+ (t = I^-+ D_oe^+ in, out = in - I^-+ D_eo^+ t)
        if (out_parity != 1) return fail(MOBIUS_EINVAL, "SCHUR_RIGHT acts on the odd parity (out_parity = 1)");
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        char *t;
        if (fixed_scratch) {
            if (2 * fb > fixed_bytes)
                return fail(MOBIUS_EINVAL, "mobius_dslash_noalloc: SCHUR_RIGHT needs " + std::to_string(2 * fb) +
                                               " bytes of workspace, above the fixed maximum of " +
                                               std::to_string(fixed_bytes));
            t = static_cast<char *>(fixed_scratch);
        } else {
            HIPCHK(ctx->scratch.ensure(2 * fb));
            t = static_cast<char *>(ctx->scratch.p);
        }
        char *v = t + fb;
        if (!dag) {
            HIPCHK(launch_m5(ctx->g, ctx->c, prec, 1, 0, in, v, nrhs, st));
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_M5INV | EPI_BMIX, 0, v, t, nullptr, nullptr, nullptr, nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_POSTSUB, 1, t, out, in, nullptr, nullptr, nrhs), st));
        } else {
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_M5INV, 0, in, t, nullptr, nullptr, nullptr, nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_M5INV | EPI_POSTSUB, 1, t, out, in, nullptr, nullptr, nrhs), st));
        }
        return MOBIUS_OK;
    }
    case MOBIUS_OP_HOP_LEFT:
    case MOBIUS_OP_SCHUR_LEFT: {
        // blocks of the left form D^ = D-^-1 D_DW D- (Sec. 2.1): hop -1/2 B H,
        // diagonal block I, Schur operator 1 - I^-1 D^_oe I^-1 D^_eo
        if (ctx->sdep) return fail(MOBIUS_EINVAL, "the left-form blocks need constant b5, c5");
        const OpCoeffs cb = b_coeffs(ctx->c, ctx->g.Ls);
        if (!std::isfinite(cb.inv_den)) return fail(MOBIUS_EINVAL, "B = b5 + c5 C5 is singular");
        const bool schur_op = op == MOBIUS_OP_SCHUR_LEFT;
        if (schur_op && out_parity != 1)
            return fail(MOBIUS_EINVAL, "SCHUR_LEFT acts on the odd parity (out_parity = 1)");
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        const int64_t need = schur_op ? 2 * fb : fb;
        char *t;
        if (fixed_scratch) {
            if (need > fixed_bytes)
                return fail(MOBIUS_EINVAL, "mobius_dslash_noalloc: the left-form operator needs " +
                                               std::to_string(need) + " bytes of workspace, above the fixed maximum of " +
                                               std::to_string(fixed_bytes));
            t = static_cast<char *>(fixed_scratch);
        } else {
            HIPCHK(ctx->scratch.ensure(need));
            t = static_cast<char *>(ctx->scratch.p);
        }
        if (!schur_op) {
            if (!dag) {  // -1/2 B H in
                HIPCHK(hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_BMIX, out_parity, in, out, nullptr, nullptr,
                                         nullptr, nrhs), st));
            } else {  // (D^_{1-p,p})^+ = -1/2 H^+ B^+
                HIPCHK(launch_m5(ctx->g, cb, prec, 0, 1, in, t, nrhs, st));
                HIPCHK(hop(ctx, hop_args(prec, 1, EPI_NOBOUT, out_parity, t, out, nullptr, nullptr, nullptr, nrhs),
                           st));
            }
            return MOBIUS_OK;
        }
        char *v = t + fb;
        if (!dag) {  // t = I^-1 B (-1/2 H in);  out = in - I^-1 B (-1/2 H t)
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_M5INV | EPI_BMIX, 0, in, t, nullptr, nullptr,
                                     nullptr, nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_M5INV | EPI_BMIX | EPI_POSTSUB, 1, t, out, in,
                                     nullptr, nullptr, nrhs), st));
        } else {  // v = B^+ I^-+ in;  t = B^+ I^-+ (-1/2 H^+ v);  out = in - (-1/2 H^+ t)
            HIPCHK(launch_m5(ctx->g, ctx->c, prec, 1, 1, in, t, nrhs, st));
            HIPCHK(launch_m5(ctx->g, cb, prec, 0, 1, t, v, nrhs, st));
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_NOBOUT | EPI_M5INV | EPI_BMIX, 0, v, t, nullptr, nullptr, nullptr,
                                     nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_NOBOUT | EPI_POSTSUB, 1, t, out, in, nullptr, nullptr, nrhs),
                       st));
        }
        return MOBIUS_OK;
    }
    case MOBIUS_OP_SCHUR_COMPLEMENT: {
        // S = I - D_oe I^-1 D_eo (t = B I^-1 D_eo in, out = I in - D_oe t);
        // S^+ = I^+ - D_eo^+ I^-+ D_oe^+ (t = I^-+ D_oe^+ in, out = I^+ in - D_eo^+ t)
        if (out_parity != 1)
            return fail(MOBIUS_EINVAL, "SCHUR_COMPLEMENT acts on the odd parity (out_parity = 1)");
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        char *t;
        if (fixed_scratch) {
            if (fb > fixed_bytes)
                return fail(MOBIUS_EINVAL, "mobius_dslash_noalloc: SCHUR_COMPLEMENT needs " + std::to_string(fb) +
                                               " bytes of workspace, above the fixed maximum of " +
                                               std::to_string(fixed_bytes));
            t = static_cast<char *>(fixed_scratch);
        } else {
            HIPCHK(ctx->scratch.ensure(fb));
            t = static_cast<char *>(ctx->scratch.p);
        }
        if (!dag) {
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_M5INV | EPI_BMIX, 0, in, t, nullptr, nullptr, nullptr, nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 0, EPI_PREMIXED | EPI_M5SUB, 1, t, out, nullptr, in, nullptr, nrhs), st));
        } else {
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_M5INV, 0, in, t, nullptr, nullptr, nullptr, nrhs), st));
            HIPCHK(hop(ctx, hop_args(prec, 1, EPI_M5SUB, 1, t, out, nullptr, in, nullptr, nrhs), st));
        }
        return MOBIUS_OK;
    }
    case MOBIUS_OP_SCHUR: {
        if (out_parity != 1) return fail(MOBIUS_EINVAL, "SCHUR acts on the odd parity (out_parity = 1)");
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        char *t;
        if (fixed_scratch) {
            if (2 * fb > fixed_bytes)
                return fail(MOBIUS_EINVAL, "mobius_dslash_noalloc: SCHUR needs " + std::to_string(2 * fb) +
                                               " bytes of workspace (two packed fields per right-hand "
                                               "side), above the fixed maximum of " +
                                               std::to_string(fixed_bytes));
            t = static_cast<char *>(fixed_scratch);
        } else {
            HIPCHK(ctx->scratch.ensure(2 * fb));
            t = static_cast<char *>(ctx->scratch.p);
        }
        HIPCHK(schur(ctx, prec, dag, in, out, t, t + fb, nullptr, nrhs, st));
        return MOBIUS_OK;
    }
    }
    return fail(MOBIUS_EINVAL, "unknown operator " + std::to_string(op));
}

}  // namespace

extern "C" int mobius_dslash(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity,
                             const void *in, void *out, int32_t nrhs, void *stream)
{
    return dslash_common(ctx, prec, op, out_parity, in, out, nrhs, stream, 0);
}

extern "C" int mobius_dslash_dag(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity,
                                 const void *in, void *out, int32_t nrhs, void *stream)
{
    return dslash_common(ctx, prec, op, out_parity, in, out, nrhs, stream, 1);
}

extern "C" int mobius_dslash_noalloc(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity,
                                     int32_t dagger, const void *in, void *out, int32_t nrhs,
                                     void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    void *ws = noalloc_scratch(ctx->device);
    if (!ws) return fail(MOBIUS_EHIP, "mobius_dslash_noalloc: no workspace on this device");
    return dslash_common(ctx, prec, op, out_parity, in, out, nrhs, stream, dagger ? 1 : 0, ws,
                         NOALLOC_SCRATCH_BYTES);
}

extern "C" int mobius_m5inv(mobius_ctx *ctx, int32_t prec, int32_t dagger, const void *in, void *out,
                            int32_t nrhs, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_prec(prec)) return r;
    if (!in || !out || nrhs < 1) return fail(MOBIUS_EINVAL, "null field or nrhs < 1");
    if (in == out) return fail(MOBIUS_EINVAL, "in and out alias");
    HIPCHK(launch_m5(ctx->g, ctx->c, prec, 1, dagger ? 1 : 0, in, out, nrhs, S(stream)));
    return MOBIUS_OK;
}

extern "C" int mobius_cg_solve(mobius_ctx *ctx, const void *src, void *sol,
                               const mobius_solve_opts *opts, mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!src || !sol || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_cg_solve");
    if (src == sol) return fail(MOBIUS_EINVAL, "source and solution alias");
    if (int r = check_prec(opts->inner_prec)) return r;
    mobius_ctx *const ctxs[1] = {ctx};
    const void *const srcs[1] = {src};
    void *const sols[1] = {sol};
    return batch_solve(ctxs, 1, srcs, sols, *opts, info, S(stream));
}

extern "C" int mobius_cg_solve_dag(mobius_ctx *ctx, const void *src, void *sol,
                                   const mobius_solve_opts *opts, mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!src || !sol || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_cg_solve_dag");
    if (src == sol) return fail(MOBIUS_EINVAL, "source and solution alias");
    if (int r = check_prec(opts->inner_prec)) return r;
    mobius_ctx *const ctxs[1] = {ctx};
    const void *const srcs[1] = {src};
    void *const sols[1] = {sol};
    return batch_solve(ctxs, 1, srcs, sols, *opts, info, S(stream), true);
}

extern "C" int mobius_batch_solve(int32_t n, mobius_ctx *const *ctxs, const void *const *src,
                                  void *const *sol, const mobius_solve_opts *opts,
                                  mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (n < 1 || !ctxs || !src || !sol || !opts || !info)
        return fail(MOBIUS_EINVAL, "bad argument to mobius_batch_solve");
    if (int r = check_prec(opts->inner_prec)) return r;
    for (int j = 0; j < n; ++j) {
        if (!ctxs[j] || !src[j] || !sol[j]) return fail(MOBIUS_EINVAL, "null context or field in batch");
        if (src[j] == sol[j]) return fail(MOBIUS_EINVAL, "source and solution alias");
        for (int k = 0; k < j; ++k)
            if (ctxs[k] == ctxs[j]) return fail(MOBIUS_EINVAL, "a context appears twice in one batch");
    }
    return batch_solve(ctxs, n, src, sol, *opts, info, S(stream));
}

extern "C" int mobius_propagator4d(mobius_ctx *ctx, const void *src4, void *sol4,
                                   const mobius_solve_opts *opts, mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!src4 || !sol4 || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_propagator4d");
    if (src4 == sol4) return fail(MOBIUS_EINVAL, "source and solution alias");
    if (int r = check_prec(opts->inner_prec)) return r;
    const int nrhs = opts->nrhs > 0 ? opts->nrhs : 1;
    hipStream_t st = S(stream);
    const Geometry &g = ctx->g;
    // temporaries: 5d source and 5d solution (canonical; the wall field lives
    // in the solution's buffer until it is packed), and the packed halves of
    // the wall field and of D(1) applied to it (FP64)
    const int64_t c5 = g.V * g.Ls * 12 * (int64_t)sizeof(double2) * nrhs;
    const int64_t fb = field_bytes(g, MOBIUS_F64) * nrhs;
    HIPCHK(ctx->prop.ensure(2 * c5 + 4 * fb));
    char *eta = static_cast<char *>(ctx->prop.p), *psi = eta + c5, *wall = psi;
    char *we = psi + c5, *wo = we + fb, *de = wo + fb, *dod = de + fb;
    HIPCHK(launch_wall_place(g, src4, wall, nrhs, st));
    HIPCHK(launch_pack_spinor(g, MOBIUS_F64, wall, we, wo, nrhs, st));
    // eta = D(1) P b: the Pauli-Villars operator (mf = 1) on the same links,
    // out_p = D_{p,1-p} in_{1-p} + I in_p for both parities
    mobius_params pv = ctx->P;
    pv.mf = 1.0;
    OpCoeffs cpv = make_coeffs(pv);
    cpv.ls = ctx->c.ls;  // per-slice coefficients do not depend on the mass
    const int32_t *nbr = static_cast<const int32_t *>(ctx->nbr.p);
    HopArgs a = hop_args(MOBIUS_F64, 0, EPI_M5ADD, 0, wo, de, nullptr, we, nullptr, nrhs);
    a.tune = &ctx->tune[MOBIUS_F64];
    HIPCHK(launch_hop(g, cpv, hop_links(ctx, MOBIUS_F64, 0), nbr, a, st));
    a = hop_args(MOBIUS_F64, 0, EPI_M5ADD, 1, we, dod, nullptr, wo, nullptr, nrhs);
    a.tune = &ctx->tune[MOBIUS_F64];
    HIPCHK(launch_hop(g, cpv, hop_links(ctx, MOBIUS_F64, 0), nbr, a, st));
    HIPCHK(launch_unpack_spinor(g, MOBIUS_F64, de, dod, eta, nrhs, st));
    // D(m) psi = eta, then q = (P^+ psi)_0
    mobius_solve_opts o = *opts;
    o.nrhs = nrhs;
    mobius_ctx *const ctxs[1] = {ctx};
    const void *const srcs[1] = {eta};
    void *const sols[1] = {psi};
    const int rc = batch_solve(ctxs, 1, srcs, sols, o, info, st);
    if (rc < 0) return rc;
    HIPCHK(launch_wall_read(g, psi, sol4, nrhs, st));
    return rc;
}

namespace {

// The Pauli-Villars (mf = 1) view of a context: the same lattice, links and
// per-slice coefficients, its own solver buffers (created on first use).
mobius_ctx *pv_view(mobius_ctx *ctx)
{
    if (ctx->pv) return ctx->pv;
    mobius_ctx *v = new mobius_ctx();
    v->P = ctx->P;
    v->P.mf = 1.0;
    v->c = make_coeffs(v->P);
    v->c.ls = ctx->c.ls;
    v->g = ctx->g;
    v->device = ctx->device;
    v->canon_of = ctx->canon_of;
    v->nbr = ctx->nbr;
    for (int q = 0; q < 3; ++q) {
        v->links[q] = ctx->links[q];
        v->links_dag[q] = ctx->links_dag[q];
        v->tune[q] = ctx->tune[q];
    }
    v->ls_coef = ctx->ls_coef;
    v->has_mu = ctx->has_mu;
    v->sdep = ctx->sdep;
    v->borrowed = true;
    ctx->pv = v;
    return v;
}

}  // namespace

extern "C" int mobius_bulk5d(mobius_ctx *ctx, const void *psi4, void *Psi5, const mobius_solve_opts *opts,
                             mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!psi4 || !Psi5 || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_bulk5d");
    if (psi4 == Psi5) return fail(MOBIUS_EINVAL, "input and output alias");
    if (int r = check_prec(opts->inner_prec)) return r;
    const int nrhs = opts->nrhs > 0 ? opts->nrhs : 1;
    hipStream_t st = S(stream);
    const Geometry &g = ctx->g;
    // temporaries: r = D(m) P psi~ and y (canonical 5d), the packed halves of
    // P psi~ and of r (FP64); P psi~ itself lives in y's buffer until packed
    const int64_t c5 = g.V * g.Ls * 12 * (int64_t)sizeof(double2) * nrhs;
    const int64_t fb = field_bytes(g, MOBIUS_F64) * nrhs;
    HIPCHK(ctx->prop.ensure(2 * c5 + 4 * fb));
    char *rr = static_cast<char *>(ctx->prop.p), *y = rr + c5, *wall = y;
    char *we = y + c5, *wo = we + fb, *re = wo + fb, *ro = re + fb;
    HIPCHK(launch_wall_place(g, psi4, wall, nrhs, st));  // P psi~ (psi~ = psi on slice 1)
    HIPCHK(launch_pack_spinor(g, MOBIUS_F64, wall, we, wo, nrhs, st));
    HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_M5ADD, 0, wo, re, nullptr, we, nullptr, nrhs), st));
    HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_M5ADD, 1, we, ro, nullptr, wo, nullptr, nrhs), st));
    HIPCHK(launch_unpack_spinor(g, MOBIUS_F64, re, ro, rr, nrhs, st));
    // D(1) y = r: the Pauli-Villars solve
    mobius_solve_opts o = *opts;
    o.nrhs = nrhs;
    mobius_ctx *const ctxs[1] = {pv_view(ctx)};
    const void *const srcs[1] = {rr};
    void *const sols[1] = {y};
    const int rc = batch_solve(ctxs, 1, srcs, sols, o, info, st);
    if (rc < 0) return rc;
    HIPCHK(launch_bulk_assemble(g, psi4, y, Psi5, nrhs, st));
    return rc;
}

extern "C" int mobius_force_lie(mobius_ctx *ctx, const void *links_c128, const void *grad_links_c128,
                                void *lie_c128, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!links_c128 || !grad_links_c128 || !lie_c128) return fail(MOBIUS_EINVAL, "null argument to mobius_force_lie");
    if (lie_c128 == links_c128 || lie_c128 == grad_links_c128)
        return fail(MOBIUS_EINVAL, "the output aliases an input");
    HIPCHK(launch_lie_force(4 * ctx->g.V, links_c128, grad_links_c128, lie_c128, S(stream)));
    return MOBIUS_OK;
}

extern "C" int mobius_force(mobius_ctx *ctx, const void *phi, void *grad_links, void *grad_phi,
                            double *action, const mobius_solve_opts *opts, mobius_solve_info *info,
                            void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!phi || !grad_phi || !action || !opts || !info)
        return fail(MOBIUS_EINVAL, "null argument to mobius_force");
    if (opts->nrhs > 1) return fail(MOBIUS_EINVAL, "mobius_force takes one source (nrhs <= 1)");
    if (int r = check_prec(opts->inner_prec)) return r;
    if (phi == grad_phi || phi == grad_links || grad_phi == grad_links)
        return fail(MOBIUS_EINVAL, "mobius_force arguments alias");
    return mobius::force(ctx, phi, grad_links, grad_phi, action, *opts, info, S(stream));
}

extern "C" int mobius_force_wall(mobius_ctx *ctx, const void *phi4, void *grad_links, double *action,
                                 const mobius_solve_opts *opts, mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!phi4 || !action || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_force_wall");
    if (opts->nrhs > 1) return fail(MOBIUS_EINVAL, "mobius_force_wall takes one source (nrhs <= 1)");
    if (int r = check_prec(opts->inner_prec)) return r;
    if (grad_links == phi4) return fail(MOBIUS_EINVAL, "mobius_force_wall arguments alias");
    hipStream_t st = S(stream);
    const Geometry &g = ctx->g;
    // temporaries: three canonical 5d fields (P phi~ then D(1) D(1)^+ chi, chi,
    // psi), the packed halves of chi, of psi and of D(1)^+ chi, norm partials
    const int64_t c5 = g.V * g.Ls * 12 * (int64_t)sizeof(double2);
    const int64_t fb = field_bytes(g, MOBIUS_F64);
    const int64_t nb = norm2_blocks(2 * fb / 8);
    HIPCHK(ctx->prop.ensure(3 * c5 + 6 * fb + (nb + 1) * (int64_t)sizeof(double)));
    char *w = static_cast<char *>(ctx->prop.p), *chi = w + c5, *psi = chi + c5;
    char *ce = psi + c5, *co = ce + fb, *pe = co + fb, *po = pe + fb, *de = po + fb, *dd = de + fb;
    double *parts = reinterpret_cast<double *>(dd + fb), *snorm = parts + nb;
    mobius_solve_opts o = *opts;
    o.nrhs = 1;
    mobius_ctx *const ctxs[1] = {ctx};
    mobius_solve_info i1{}, i2{};
    // chi = D(m)^-+ P phi~
    HIPCHK(launch_wall_place(g, phi4, w, 1, st));
    {
        const void *const srcs[1] = {w};
        void *const sols[1] = {chi};
        const int rc = batch_solve(ctxs, 1, srcs, sols, o, &i1, st, true);
        if (rc < 0) return rc;
    }
    // d = D(1)^+ chi, then w = D(1) d (the Pauli-Villars operator on the same links)
    mobius_params pvp = ctx->P;
    pvp.mf = 1.0;
    OpCoeffs cpv = make_coeffs(pvp);
    cpv.ls = ctx->c.ls;
    const int32_t *nbr = static_cast<const int32_t *>(ctx->nbr.p);
    HIPCHK(launch_pack_spinor(g, MOBIUS_F64, chi, ce, co, 1, st));
    for (int dag = 1; dag >= 0; --dag) {
        const char *ie = dag ? ce : de, *io = dag ? co : dd;
        char *oe = dag ? de : pe, *oo = dag ? dd : po;
        HopArgs a = hop_args(MOBIUS_F64, dag, EPI_M5ADD, 0, io, oe, nullptr, ie, nullptr, 1);
        a.tune = &ctx->tune[MOBIUS_F64];
        HIPCHK(launch_hop(g, cpv, hop_links(ctx, MOBIUS_F64, dag), nbr, a, st));
        a = hop_args(MOBIUS_F64, dag, EPI_M5ADD, 1, ie, oo, nullptr, io, nullptr, 1);
        a.tune = &ctx->tune[MOBIUS_F64];
        HIPCHK(launch_hop(g, cpv, hop_links(ctx, MOBIUS_F64, dag), nbr, a, st));
    }
    HIPCHK(launch_norm2_f64(reinterpret_cast<const double *>(de), 2 * fb / 8, parts, snorm, st));  // S = |d|^2
    HIPCHK(launch_unpack_spinor(g, MOBIUS_F64, pe, po, w, 1, st));
    // psi = D(m)^-1 D(1) D(1)^+ chi
    {
        const void *const srcs[1] = {w};
        void *const sols[1] = {psi};
        const int rc = batch_solve(ctxs, 1, srcs, sols, o, &i2, st, false);
        if (rc < 0) return rc;
    }
    if (grad_links) {
        // G = -G[chi, psi; m] + G[chi, d; 1], G[L, R; c] the gradient of 2 Re <L, dD_hop R>
        HIPCHK(launch_pack_spinor(g, MOBIUS_F64, psi, pe, po, 1, st));
        for (int par = 0; par < 2; ++par) {
            const char *Lp = par ? co : ce, *Ln = par ? ce : co;
            HIPCHK(launch_force(g, ctx->c, par, nbr, Lp, par ? po : pe, Ln, par ? pe : po, grad_links, st,
                                -1.0, false, ctx->P.mu));
            HIPCHK(launch_force(g, cpv, par, nbr, Lp, par ? dd : de, Ln, par ? de : dd, grad_links, st,
                                1.0, true, ctx->P.mu));
        }
    }
    HIPCHK(hipMemcpyAsync(action, snorm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // one record for the pair of solves: iterations and Dirac applications
    // summed, the worse residual, the larger condition number
    *info = i2;
    info->iters = i1.iters + i2.iters;
    info->dirac_apps = i1.dirac_apps + i2.dirac_apps + 4;
    info->reliable_updates = i1.reliable_updates + i2.reliable_updates;
    info->status = (i1.status == MOBIUS_OK && i2.status == MOBIUS_OK) ? MOBIUS_OK : MOBIUS_NOT_CONVERGED;
    info->true_resid = std::max(i1.true_resid, i2.true_resid);
    info->schur_resid = std::max(i1.schur_resid, i2.schur_resid);
    info->seconds = i1.seconds + i2.seconds;
    info->algo_bytes = i1.algo_bytes + i2.algo_bytes;
    info->flops = i1.flops + i2.flops;
    info->kappa = std::max(i1.kappa, i2.kappa);
    info->err_bound = std::max(i1.err_bound, i2.err_bound);
    return info->status;
}

extern "C" int mobius_tune(mobius_ctx *ctx, int32_t prec, int32_t reps, mobius_tune_result *out,
                           void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (int r = check_prec(prec)) return r;
    return mobius::tune(ctx, prec, reps, out, S(stream));
}

extern "C" int mobius_tune_brick(const mobius_params *p, const void *links_c128, int32_t prec,
                                 int32_t reps, mobius_brick_trial *trials, int32_t max_trials,
                                 int32_t *ntrials, int32_t *brick_out, double *us_out, void *stream)
{
    g_err.clear();
    if (!p || !links_c128 || !brick_out) return fail(MOBIUS_EINVAL, "null argument to mobius_tune_brick");
    if (int r = check_prec(prec)) return r;
    if (trials && max_trials < 0) return fail(MOBIUS_EINVAL, "max_trials must be >= 0");
    for (int mu = 0; mu < 4; ++mu)
        if (p->L[mu] < 2 || (p->L[mu] & 1))
            return fail(MOBIUS_EINVAL, "every lattice extent must be even and >= 2");
    if (p->Ls < 2 || p->Ls > 64) return fail(MOBIUS_EINVAL, "Ls must be in [2, 64]");
    int base[3];
    choose_brick(p->L, p->Ls, base);
    // candidates: each side kept, halved or doubled (side k of candidate i
    // by the k-th base-3 digit of i; i = 0 is the automatic brick) where it
    // still divides the lattice
    struct Cand {
        int b[3];
        double dist, surf;
    };
    std::vector<Cand> cands;
    const double vol0 = (double)base[0] * base[1] * base[2];
    for (int i = 0; i < 27; ++i) {
        Cand c;
        int f = i;
        bool ok = true;
        for (int k = 0; k < 3; ++k, f /= 3) {
            const int s = f % 3 == 0 ? base[k] : f % 3 == 1 ? base[k] / 2 : base[k] * 2;
            // (the automatic brick itself is always a candidate, also an
            // override that does not divide the lattice)
            ok = ok && (i == 0 || (s >= 1 && s <= p->L[k] && p->L[k] % s == 0 && (f % 3 != 1 || base[k] % 2 == 0)));
            c.b[k] = s;
        }
        if (!ok) continue;
        bool dup = false;
        for (const Cand &d : cands) dup = dup || (d.b[0] == c.b[0] && d.b[1] == c.b[1] && d.b[2] == c.b[2]);
        if (dup) continue;
        c.dist = std::fabs(std::log2((double)c.b[0] * c.b[1] * c.b[2] / vol0));
        c.surf = 1.0 / c.b[0] + 1.0 / c.b[1] + 1.0 / c.b[2];
        cands.push_back(c);
    }
    // the automatic brick first (i = 0), then nearest in volume, then most compact
    std::stable_sort(cands.begin() + 1, cands.end(), [](const Cand &x, const Cand &y) {
        return x.dist != y.dist ? x.dist < y.dist : x.surf < y.surf;
    });
    if (cands.size() > 12) cands.resize(12);
    int best = 0;
    double best_us = 0, base_us = 0;
    int n = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        mobius_params q = *p;
        for (int k = 0; k < 3; ++k) q.brick[k] = cands[i].b[k];
        mobius_ctx *ctx = nullptr;
        if (int r = mobius_create(&ctx, &q, links_c128, stream)) return r;
        mobius_tune_result res;
        const int r = mobius::tune(ctx, prec, reps, &res, S(stream));
        mobius_destroy(ctx);
        if (r != MOBIUS_OK) return r;
        if (trials && n < max_trials) {
            for (int k = 0; k < 3; ++k) trials[n].brick[k] = cands[i].b[k];
            trials[n].hop_us = res.hop_us;
        }
        ++n;
        if (i == 0) {
            base_us = best_us = res.hop_us;
        } else if (res.hop_us < best_us && res.hop_us < 0.97 * base_us) {
            best = (int)i;
            best_us = res.hop_us;
        }
    }
    for (int k = 0; k < 3; ++k) brick_out[k] = cands[best].b[k];
    if (us_out) *us_out = best_us;
    if (ntrials) *ntrials = trials ? std::min(n, (int)max_trials) : n;
    return MOBIUS_OK;
}

extern "C" int mobius_set_tuning(mobius_ctx *ctx, const mobius_tune_result *t)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!t) return fail(MOBIUS_EINVAL, "null tuning");
    if (int r = check_prec(t->prec)) return r;
    if (t->prefetch < 0 || t->prefetch > 2 || (t->stage_links & ~1) || (t->xcd_remap & ~1) ||
        (t->nt_links & ~1) || (t->mfma & ~1))
        return fail(MOBIUS_EINVAL, "tuning value out of range");
    HopTuning h;
    h.prefetch = t->prefetch;
    h.stage_links = t->stage_links;
    h.xcd_remap = t->xcd_remap;
    h.nt_links = t->nt_links;
    h.mfma = t->mfma;
    ctx->tune[t->prec] = h;
    ctx->tuned_us[t->prec] = 0;
    return MOBIUS_OK;
}
