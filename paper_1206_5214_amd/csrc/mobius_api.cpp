// mobius_api.cpp -- C ABI of libmobius.so: context, red/black operator blocks
// and the CGLS solvers (plain FP64, and low-precision operator with FP64
// reductions, reliable updates and outer defect correction).
#include "mobius_internal.h"

#include <hip/hip_runtime.h>

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

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MOBIUS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

// device buffer owned by the context
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

}  // namespace

struct mobius_ctx {
    mobius_params P{};
    Geometry g{};
    OpCoeffs c{};
    int device = 0;
    DevBuf canon_of;     // [2][Vh] canonical index of each packed site
    DevBuf nbr;
    DevBuf links[3];
    DevBuf scratch;      // operator temporaries (SCHUR blocks)
    DevBuf work;         // solver fields
    DevBuf partials;     // reduction partials
    DevBuf scalars;      // CgScalars + extra doubles
};

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
    return c;
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

// MOBIUS_DEBUG=1 prints the CG scalars of every iteration to stderr.
int debug_level()
{
    static const int lvl = [] {
        const char *e = std::getenv("MOBIUS_DEBUG");
        return e ? std::atoi(e) : 0;
    }();
    return lvl;
}

// Reduction workspace large enough for a hop-kernel norm and a BLAS norm.
int ensure_partials(mobius_ctx *ctx, int nrhs)
{
    int64_t n = std::max(site_kernel_blocks(ctx->g), blas_blocks(ctx->g)) * std::max(nrhs, 1);
    HIPCHK(ctx->partials.ensure(n * (int64_t)sizeof(double)));
    HIPCHK(ctx->scalars.ensure(64 * (int64_t)sizeof(double) * std::max(nrhs, 1)));
    return MOBIUS_OK;
}

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
// x Ls x 192 B) stays within 1 MiB, i.e. a few slices fit one XCD's 4 MiB L2;
// ties go to the smaller surface.
void choose_brick(const int L[4], int Ls, int brick[3])
{
    if (const char *e = std::getenv("MOBIUS_BRICK")) {
        int b[3];
        if (std::sscanf(e, "%d,%d,%d", &b[0], &b[1], &b[2]) == 3 && b[0] > 0 && b[1] > 0 && b[2] > 0) {
            for (int k = 0; k < 3; ++k) brick[k] = std::min(b[k], L[k]);
            return;
        }
    }
    const double budget = 1024.0 * 1024.0;
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
    const double Mp = p->b5 * (4.0 - p->M5) + 1.0;
    if (Mp == 0.0) return fail(MOBIUS_EINVAL, "M+ = b5 (4 - M5) + 1 is zero");
    const OpCoeffs c = make_coeffs(*p);
    if (!std::isfinite(c.inv_den)) return fail(MOBIUS_EINVAL, "the Ls-direction block I is singular");

    mobius_ctx *ctx = new mobius_ctx();
    ctx->P = *p;
    ctx->c = c;
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
    // site order and neighbour table
    choose_brick(g.L, g.Ls, g.brick);
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
        e = ctx->links[prec].ensure(2 * 8 * g.Vh * (int64_t)link_record_bytes(prec));
        if (e != hipSuccess) return cleanup(fail(MOBIUS_ENOMEM, "links: " + std::string(hipGetErrorString(e))));
        e = launch_pack_links(g, prec, links_c128, ctx->links[prec].p, st);
        if (e != hipSuccess) return cleanup(fail(MOBIUS_EHIP, hipGetErrorString(e)));
    }
    *out = ctx;
    return MOBIUS_OK;
}

extern "C" int mobius_destroy(mobius_ctx *ctx)
{
    if (!ctx) return MOBIUS_OK;
    (void)hipDeviceSynchronize();
    ctx->nbr.release();
    ctx->canon_of.release();
    for (auto &l : ctx->links) l.release();
    ctx->scratch.release();
    ctx->work.release();
    ctx->partials.release();
    ctx->scalars.release();
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

hipError_t hop(mobius_ctx *ctx, const HopArgs &a, hipStream_t st)
{
    return launch_hop(ctx->g, ctx->c, ctx->links[a.prec].p, static_cast<const int32_t *>(ctx->nbr.p),
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
        // t = I^-1 D_eo in ;  out = in - I^-1 D_oe t
        e = hop(ctx, hop_args(prec, 0, EPI_M5INV, 0, in, t_even, nullptr, nullptr, nullptr, nrhs), st);
        if (e != hipSuccess) return e;
        return hop(ctx, hop_args(prec, 0, EPI_M5INV | EPI_POSTSUB | norm, 1, t_even, out, in,
                                 nullptr, partials, nrhs), st);
    }
    // u = I^-+ in ;  t = I^-+ (D_oe)^+ u ;  out = in - (D_eo)^+ t
    e = launch_m5(ctx->g, ctx->c, prec, 1, 1, in, u_odd, nrhs, st);
    if (e != hipSuccess) return e;
    e = hop(ctx, hop_args(prec, 1, EPI_M5INV, 0, u_odd, t_even, nullptr, nullptr, nullptr, nrhs), st);
    if (e != hipSuccess) return e;
    return hop(ctx, hop_args(prec, 1, EPI_POSTSUB | norm, 1, t_even, out, in, nullptr, partials, nrhs),
               st);
}

int dslash_common(mobius_ctx *ctx, int32_t prec, int32_t op, int32_t out_parity, const void *in,
                  void *out, int32_t nrhs, void *stream, int dag)
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
    case MOBIUS_OP_SCHUR: {
        if (out_parity != 1) return fail(MOBIUS_EINVAL, "SCHUR acts on the odd parity (out_parity = 1)");
        const int64_t fb = field_bytes(ctx->g, prec) * nrhs;
        HIPCHK(ctx->scratch.ensure(2 * fb));
        char *t = static_cast<char *>(ctx->scratch.p);
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

// ---------------------------------------------------------------------------
// Solver

namespace {

__global__ void set_scalar_kernel(double *p, double v) { *p = v; }

struct Solver {
    mobius_ctx *ctx;
    hipStream_t st;
    const Geometry &g;
    int lo;                  // precision of the CG operator and Krylov vectors
    int px;                  // precision of the solution correction x (FP32 when lo is FP16)
    int64_t fb64 = 0, fblo = 0, fbx = 0;
    // FP64 fields: packed source, b', x_hi, r_hi, temporaries, even half of psi
    char *eta_e, *eta_o, *b, *xh, *rh, *t64, *u64, *q64, *pe;
    // CG fields in precision lo
    char *x, *r, *p, *q, *s, *t, *u;
    double *part;
    CgScalars *sc;
    double *extra;           // device doubles: [0] |b|^2 [2],[3] |true res|^2 (e,o) [4] |r_hi|^2
                             // [5],[6] |eta_e|^2,|eta_o|^2 [8] = -1
    int dirac = 0;
    double abytes = 0, aflops = 0;  // algorithmic HBM bytes and flops of the launches

    // -- accounting (per launch, per the conventions in mobius.h) -----------
    double fbd(int prec) const { return (double)field_bytes(g, prec); }
    double N5d() const { return (double)g.N5; }
    void acct_hop(int prec, int epi)
    {
        abytes += 2 * fbd(prec) + 72.0 * g.Vh * link_elem_bytes(prec);  // 9 complex per link
        aflops += 1416 * N5d();
        if (epi & (EPI_PRESUB | EPI_POSTSUB)) { abytes += fbd(prec); aflops += 24 * N5d(); }
        if (epi & EPI_M5ADD) { abytes += fbd(prec); aflops += 96 * N5d(); }
        if (epi & EPI_M5INV) aflops += 96 * N5d();
        if (epi & EPI_NORM) aflops += 48 * N5d();
    }
    void acct_m5(int prec) { abytes += 2 * fbd(prec); aflops += 96 * N5d(); }
    void acct_vec(double nbytes, double nflops) { abytes += nbytes; aflops += nflops * N5d(); }

    Solver(mobius_ctx *c, hipStream_t s_, int prec)
        : ctx(c), st(s_), g(c->g), lo(prec), px(prec == MOBIUS_F16 ? MOBIUS_F32 : prec)
    {
    }

    static int64_t bytes_needed(const Geometry &g, int prec)
    {
        const int px = prec == MOBIUS_F16 ? MOBIUS_F32 : prec;
        return 9 * field_bytes(g, MOBIUS_F64) + 6 * field_bytes(g, prec) + field_bytes(g, px) + 4096;
    }

    int allocate()
    {
        fb64 = field_bytes(g, MOBIUS_F64);
        fblo = field_bytes(g, lo);
        fbx = field_bytes(g, px);
        HIPCHK(ctx->work.ensure(bytes_needed(g, lo)));
        char *w = static_cast<char *>(ctx->work.p);
        char **hi[9] = {&eta_e, &eta_o, &b, &xh, &rh, &t64, &u64, &q64, &pe};
        for (int k = 0; k < 9; ++k) {
            *hi[k] = w;
            w += fb64;
        }
        x = w;
        w += fbx;
        char **lf[6] = {&r, &p, &q, &s, &t, &u};
        for (int k = 0; k < 6; ++k) {
            *lf[k] = w;
            w += fblo;
        }
        if (int rc = ensure_partials(ctx, 1)) return rc;
        part = static_cast<double *>(ctx->partials.p);
        sc = static_cast<CgScalars *>(ctx->scalars.p);
        extra = reinterpret_cast<double *>(sc + 1);
        return MOBIUS_OK;
    }

    int64_t hop_nb() const { return site_kernel_blocks(g); }
    int64_t blas_nb() const { return blas_blocks(g); }

    // out = D_pre in (dag = 0) or D_pre^+ in (dag = 1); |out|^2 -> *dst if dst
    hipError_t apply(int prec, int dag, const void *in, void *out, void *tt, void *uu, double *dst)
    {
        dirac += 2;
        const int norm = dst ? EPI_NORM : 0;
        if (!dag) {
            acct_hop(prec, EPI_M5INV);
            acct_hop(prec, EPI_M5INV | EPI_POSTSUB | norm);
        } else {
            acct_m5(prec);
            acct_hop(prec, EPI_M5INV);
            acct_hop(prec, EPI_POSTSUB | norm);
        }
        hipError_t e = schur(ctx, prec, dag, in, out, tt, uu, dst ? part : nullptr, 1, st);
        if (e != hipSuccess || !dst) return e;
        return launch_reduce(part, hop_nb(), dst, st);
    }
    hipError_t norm2(int prec, const void *f, double *dst)
    {
        acct_vec(fbd(prec), 48);
        hipError_t e = launch_norm2(g, prec, f, part, 1, st);
        if (e != hipSuccess) return e;
        return launch_reduce(part, blas_nb(), dst, st);
    }
    int fetch(double *host, const double *dev, int n)
    {
        HIPCHK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return MOBIUS_OK;
    }
    // r_hi = b - D_pre x_hi in FP64, |r_hi|^2 -> extra[4]
    hipError_t true_schur_residual()
    {
        hipError_t e = apply(MOBIUS_F64, 0, xh, q64, t64, u64, nullptr);
        if (e != hipSuccess) return e;
        e = launch_axpby(g, MOBIUS_F64, nullptr, b, extra + 8, q64, rh, 1, st);
        if (e != hipSuccess) return e;
        acct_vec(3 * fbd(MOBIUS_F64), 48);
        return norm2(MOBIUS_F64, rh, extra + 4);
    }

    int solve_one(const void *src, void *sol, const mobius_solve_opts &o, mobius_solve_info &info);
};

// CGLS on D_pre (odd parity) for D_DW psi = eta, red/black decomposition of
// Sec. 3.  With lo = F64 this is plain FP64 CGLS; with lo = F32/F16 the
// operator and Krylov vectors are low precision, every norm and inner
// product is an FP64 reduction, x is accumulated in FP64, and the residual is
// replaced by the FP64 true residual b - D_pre x whenever |r| has fallen by
// `delta` since the last replacement (reliable update).  When a replacement
// does not reduce the true residual by at least 2x the Krylov space is
// restarted from it (defect correction).  The stopping test is on the FP64
// true residual of the full system after reconstruction.
int Solver::solve_one(const void *src, void *sol, const mobius_solve_opts &o,
                      mobius_solve_info &info)
{
    const double tol = o.tol > 0 ? o.tol : 1e-10;
    const int maxiter = o.maxiter > 0 ? o.maxiter : 10000;
    const int check = o.check_every > 0 ? o.check_every : 16;
    const bool mixed = lo != MOBIUS_F64;
    const double delta = mixed ? (o.reliable_delta > 0 ? o.reliable_delta : 0.1) : 0.0;
    dirac = 0;
    abytes = aflops = 0;
    std::memset(&info, 0, sizeof(info));
    const double canon_bytes = 2.0 * g.N5 * 12 * 16;

    hipEvent_t ev0, ev1;
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, st));
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(1), 0, st, extra + 8, -1.0);
    HIPCHK(hipGetLastError());

    // pack the source; b' = I^-1 (eta_o - D_oe I^-1 eta_e)
    HIPCHK(launch_pack_spinor(g, MOBIUS_F64, src, eta_e, eta_o, 1, st));
    acct_vec(canon_bytes + 2 * fbd(MOBIUS_F64), 0);
    HIPCHK(launch_m5(g, ctx->c, MOBIUS_F64, 1, 0, eta_e, t64, 1, st));
    acct_m5(MOBIUS_F64);
    HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_PRESUB | EPI_M5INV, 1, t64, b, eta_o), st));
    acct_hop(MOBIUS_F64, EPI_PRESUB | EPI_M5INV);
    dirac += 1;
    HIPCHK(norm2(MOBIUS_F64, b, extra + 0));
    HIPCHK(norm2(MOBIUS_F64, eta_e, extra + 5));
    HIPCHK(norm2(MOBIUS_F64, eta_o, extra + 6));
    double hb[8];
    if (int rc = fetch(hb, extra, 8)) return rc;
    const double bnorm2 = hb[0];
    const double etanorm = std::sqrt(hb[5] + hb[6]);

    // x_hi = 0, r_hi = b, x = 0, r = r_hi
    HIPCHK(launch_zero(xh, fb64, st));
    HIPCHK(launch_convert(g, MOBIUS_F64, b, MOBIUS_F64, rh, st));
    HIPCHK(launch_zero(x, fbx, st));
    HIPCHK(launch_convert(g, MOBIUS_F64, rh, lo, r, st));
    acct_vec(fbd(MOBIUS_F64) * 4 + fbd(px) + fbd(lo), 0);

    int iters = 0, reliable = 0;
    double tol_s = tol;  // relative Schur-residual target, tightened if the true residual misses
    double true_res = INFINITY, schur_res = INFINITY;
    bool converged = bnorm2 == 0.0;
    if (converged) true_res = schur_res = 0.0;

    while (!converged && iters < maxiter) {
        // (re)start the Krylov space: s = D^+ r, p = s, gamma = |s|^2
        HIPCHK(apply(lo, 1, r, s, t, u, &sc->gamma));
        HIPCHK(launch_convert(g, lo, s, lo, p, st));
        acct_vec(2 * fbd(lo), 0);
        double rmax2;
        HIPCHK(norm2(lo, r, &sc->rr));
        if (int rc = fetch(&rmax2, &sc->rr, 1)) return rc;
        bool restart = false;
        int since_check = 0;
        while (iters < maxiter) {
            HIPCHK(apply(lo, 0, p, q, t, u, &sc->qq));
            HIPCHK(launch_cg_scalar(sc, 0, st));
            HIPCHK(launch_cg_xr(g, lo, px, &sc->alpha, x, p, r, q, part, st));
            acct_vec(2 * fbd(px) + 4 * fbd(lo), 96 + 48);
            HIPCHK(launch_reduce(part, blas_nb(), &sc->rr, st));
            ++iters;
            if (debug_level() > 0) {
                CgScalars h;
                HIPCHK(hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                std::fprintf(stderr, "[mobius cg] it %d gamma %.6e qq %.6e alpha %.6e rr %.6e beta %.6e\n",
                             iters, h.gamma, h.qq, h.alpha, h.rr, h.beta);
            }
            if (mixed || ++since_check >= check || iters >= maxiter) {
                since_check = 0;
                double rr;
                if (int rc = fetch(&rr, &sc->rr, 1)) return rc;
                if (!std::isfinite(rr)) return fail(MOBIUS_EHIP, "CG breakdown: non-finite residual");
                const bool small = rr <= tol_s * tol_s * bnorm2;
                if (small || iters >= maxiter || (mixed && rr < delta * delta * rmax2)) {
                    // x_hi += x; x = 0; r_hi = b - D_pre x_hi (FP64); r = r_hi
                    HIPCHK(launch_accumulate(g, px, x, xh, st));
                    HIPCHK(launch_zero(x, fbx, st));
                    acct_vec(fbd(px) * 2 + 2 * fbd(MOBIUS_F64), 24);
                    HIPCHK(true_schur_residual());
                    double hr;
                    if (int rc = fetch(&hr, extra + 4, 1)) return rc;
                    HIPCHK(launch_convert(g, MOBIUS_F64, rh, lo, r, st));
                    acct_vec(fbd(MOBIUS_F64) + fbd(lo), 0);
                    if (mixed) ++reliable;
                    const double prev = rmax2;
                    rmax2 = hr;
                    if (hr <= tol_s * tol_s * bnorm2 || iters >= maxiter) break;
                    if (!mixed || hr > 0.25 * prev) {
                        restart = true;
                        break;
                    }
                }
            }
            HIPCHK(apply(lo, 1, r, s, t, u, &sc->gamma_new));
            HIPCHK(launch_cg_scalar(sc, 1, st));
            HIPCHK(launch_axpby(g, lo, nullptr, s, &sc->beta, p, p, 1, st));
            acct_vec(3 * fbd(lo), 48);
        }
        if (restart) continue;
        // reconstruct psi_e = I^-1 (eta_e - D_eo psi_o); FP64 true residual of D_DW psi = eta
        HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_PRESUB | EPI_M5INV, 0, xh, pe, eta_e), st));
        HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_M5ADD | EPI_PRESUB | EPI_NORM, 0, xh, t64, eta_e,
                                 pe, part), st));
        HIPCHK(launch_reduce(part, hop_nb(), extra + 2, st));
        HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_M5ADD | EPI_PRESUB | EPI_NORM, 1, pe, q64, eta_o,
                                 xh, part), st));
        HIPCHK(launch_reduce(part, hop_nb(), extra + 3, st));
        acct_hop(MOBIUS_F64, EPI_PRESUB | EPI_M5INV);
        acct_hop(MOBIUS_F64, EPI_M5ADD | EPI_PRESUB | EPI_NORM);
        acct_hop(MOBIUS_F64, EPI_M5ADD | EPI_PRESUB | EPI_NORM);
        dirac += 3;
        double h[5];
        if (int rc = fetch(h, extra, 5)) return rc;
        schur_res = std::sqrt(h[4] / bnorm2);
        true_res = etanorm > 0 ? std::sqrt(h[2] + h[3]) / etanorm : 0.0;
        if (true_res <= tol) {
            converged = true;
            break;
        }
        // tighten the Schur target and continue from x_hi (r already = r_hi)
        tol_s *= std::max(0.05, 0.5 * tol / true_res);
    }
    if (bnorm2 == 0.0) {
        HIPCHK(launch_zero(xh, fb64, st));
        HIPCHK(launch_m5(g, ctx->c, MOBIUS_F64, 1, 0, eta_e, pe, 1, st));
    } else if (!converged) {
        HIPCHK(hop(ctx, hop_args(MOBIUS_F64, 0, EPI_PRESUB | EPI_M5INV, 0, xh, pe, eta_e), st));
    }
    HIPCHK(launch_unpack_spinor(g, MOBIUS_F64, pe, xh, sol, 1, st));
    acct_vec(canon_bytes + 2 * fbd(MOBIUS_F64), 0);
    HIPCHK(hipEventRecord(ev1, st));
    HIPCHK(hipEventSynchronize(ev1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    info.iters = iters;
    info.dirac_apps = dirac;
    info.reliable_updates = reliable;
    info.status = converged ? MOBIUS_OK : MOBIUS_NOT_CONVERGED;
    info.true_resid = true_res;
    info.schur_resid = schur_res;
    info.seconds = ms * 1e-3;
    info.algo_bytes = abytes;
    info.flops = aflops;
    return info.status;
}

}  // namespace

extern "C" int mobius_cg_solve(mobius_ctx *ctx, const void *src, void *sol,
                               const mobius_solve_opts *opts, mobius_solve_info *info, void *stream)
{
    g_err.clear();
    if (int r = check_ctx(ctx)) return r;
    if (!src || !sol || !opts || !info) return fail(MOBIUS_EINVAL, "null argument to mobius_cg_solve");
    if (src == sol) return fail(MOBIUS_EINVAL, "source and solution alias");
    if (int r = check_prec(opts->inner_prec)) return r;
    const int nrhs = opts->nrhs > 0 ? opts->nrhs : 1;
    Solver sv(ctx, S(stream), opts->inner_prec);
    if (int rc = sv.allocate()) return rc;
    const int64_t canon_bytes = 2 * ctx->g.N5 * 12 * 16;
    int status = MOBIUS_OK;
    for (int k = 0; k < nrhs; ++k) {
        const char *sk = static_cast<const char *>(src) + k * canon_bytes;
        char *xk = static_cast<char *>(sol) + k * canon_bytes;
        int rc = sv.solve_one(sk, xk, *opts, info[k]);
        if (rc < 0) return rc;
        if (rc == MOBIUS_NOT_CONVERGED) status = MOBIUS_NOT_CONVERGED;
    }
    return status;
}
