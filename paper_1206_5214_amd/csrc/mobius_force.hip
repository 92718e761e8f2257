// mobius_force.hip -- link derivative of the pseudofermion action
//   S = phi^+ (D_pre^+ D_pre)^-1 phi,   D_pre = 1 - I^-1 D_oe I^-1 D_eo  (Sec. 3)
// for gfx950.
//
// With X = (D_pre^+ D_pre)^-1 phi, Y = D_pre X, Yt = I^-+ Y, Z = I^-1 D_eo X and
// W = I^-+ (D_oe)^+ Yt, a change of the links changes S by
//   dS = -Re <Yt, dH_oe (B Z)> - Re <W, dH_eo (B X)>
// (the off-diagonal blocks are D_{p,1-p} = -1/2 H_{p,1-p} B and hold all of the
// link dependence).  Write L_p for the left field of parity p (L_1 = Yt,
// L_0 = W) and R_p for the right one (R_1 = X, R_0 = Z).  The link U_mu(y),
// y of parity p, enters H at the row y (forward hop from y + mu) and at the
// row y + mu (backward hop from y), so its gradient
// G = dS/dRe U + i dS/dIm U is
//   G_ab = - sum_s sum_{spin} [ L_p(y)_a conj(((1 - g_mu) B R_{1-p}(y+mu))_b)
//                              + ((1 + g_mu) B R_p(y))_a conj(L_{1-p}(y+mu)_b) ].
// (1 + sigma g_mu)/2 is a rank-2 projector whose image is parametrised by the
// half spinor h = u + sigma A_mu l (spins 0,1), and A_mu is unitary, so each
// spin sum collapses onto the two rows of the half spinors:
//   sum_spin x_a conj(((1 + sigma g_mu) y)_b) = sum_{t=0,1} h^sigma(x)_{t,a} conj(h^sigma(y)_{t,b}).
//
// With a chemical potential the time-like forward hop carries e^{+mu} and the
// backward one e^{-mu} (on U_4(y) and U_4(y)^+), so the two terms of G for
// mu = t are weighted by those factors.
//
// Thread mapping as in the hop kernel: one lane per (site y, s), the Ls lanes
// of a site in one wavefront, B applied by cross-lane shuffles, and the sum
// over s through LDS; one launch per parity p covers the four links U_mu(y)
// of every site y of that parity.
#include "mobius_device.h"

#include <hip/hip_runtime.h>

#include <cmath>

namespace mobius {
namespace {

// half spinor h = u + sigma A_mu l of a full spinor (rows 0, 1; 3 colours each)
template <int MU, int SIGMA>
__device__ __forceinline__ void half_of(const cx<double> v[12], cx<double> h[6])
{
    const double sg = (double)SIGMA;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<double> o0, o1;
        A_apply<double, MU>(v[6 + a], v[9 + a], o0, o1);
        h[a] = v[a] + sg * o0;
        h[3 + a] = v[3 + a] + sg * o1;
    }
}

struct ForceLds {
    static constexpr int STRIDE = 9;  // complex per lane
    cx<double> buf[WAVES][64 * STRIDE];
};

// Contribution of one lane (one s) to G_mu(y), summed over s in LDS and
// written by lanes s = 0..8 (one matrix element each, or several if Ls < 9).
template <int MU>
__device__ __forceinline__ void force_dir(const ForceParams &fp, const SiteMap &m, const Coef<double> &k,
                                          const cx<double> Lo[12], const cx<double> BRo[12],
                                          uint32_t jn, ForceLds &lds)
{
    using S = Spin<MOBIUS_F64>;
    const uint32_t N5 = (uint32_t)fp.N5;
    const int64_t fb = S::bytes(fp.N5);
    cx<double> Ln[12], Rn[12];
    S::load(Buf(fp.Ln, fb), N5, jn, Ln);
    S::load(Buf(fp.Rn, fb), N5, jn, Rn);
    mix_s(Rn, mix_w(k, false, m, fp.Ls, false), k.mf, m, fp.Ls, false);  // B R_{1-p}(y + mu)

    cx<double> hL[6], hR[6], c[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) c[e] = {0, 0};
    // forward term: L_p(y) against (1 - g_mu) B R_{1-p}(y + mu)
    half_of<MU, -1>(Lo, hL);
    half_of<MU, -1>(Rn, hR);
    if constexpr (MU == 3) {
#pragma unroll
        for (int q = 0; q < 6; ++q) hR[q] = fp.ef * hR[q];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) c[a * 3 + b] = cjmadd(c[a * 3 + b], hR[t * 3 + b], hL[t * 3 + a]);
    // backward term: (1 + g_mu) B R_p(y) against L_{1-p}(y + mu)
    half_of<MU, +1>(BRo, hR);
    half_of<MU, +1>(Ln, hL);
    if constexpr (MU == 3) {
#pragma unroll
        for (int q = 0; q < 6; ++q) hR[q] = fp.eb * hR[q];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) c[a * 3 + b] = cjmadd(c[a * 3 + b], hL[t * 3 + b], hR[t * 3 + a]);

    cx<double> *w = lds.buf[m.wave];
    constexpr int ST = ForceLds::STRIDE;
#pragma unroll
    for (int e = 0; e < 9; ++e) w[m.lane * ST + e] = c[e];
    __syncthreads();
    if (m.site_ok) {
        const int base = m.g * fp.Ls;
        const int64_t link = (int64_t)MU * fp.V + fp.canon_of[m.i];
        for (int e = m.s; e < 9; e += fp.Ls) {
            cx<double> acc = {0, 0};
            for (int t = 0; t < fp.Ls; ++t) acc = acc + w[(base + t) * ST + e];
            double2 gv = make_double2(-fp.scale * acc.r, -fp.scale * acc.i);
            if (fp.accumulate) {
                const double2 old = fp.grad[link * 9 + e];
                gv = make_double2(old.x + gv.x, old.y + gv.y);
            }
            fp.grad[link * 9 + e] = gv;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(BLOCK) void force_kernel(ForceParams fp)
{
    using S = Spin<MOBIUS_F64>;
    const SiteMap m = site_map(fp.Ls, fp.spw, fp.Vh);
    const Coef<double> k = make_coef<double>(fp.c);
    const uint32_t N5 = (uint32_t)fp.N5;
    const int64_t fb = S::bytes(fp.N5);
    const uint32_t k5 = (uint32_t)m.i * (uint32_t)fp.Ls + (uint32_t)m.s;
    cx<double> Lo[12], BRo[12];
    S::load(Buf(fp.Lp, fb), N5, k5, Lo);
    S::load(Buf(fp.Rp, fb), N5, k5, BRo);
    mix_s(BRo, mix_w(k, false, m, fp.Ls, false), k.mf, m, fp.Ls, false);  // B R_p(y)
    const int32_t *nb = fp.nbr + m.i * 8;
    __shared__ ForceLds lds;
    force_dir<0>(fp, m, k, Lo, BRo, (uint32_t)nb[0] * (uint32_t)fp.Ls + (uint32_t)m.s, lds);
    force_dir<1>(fp, m, k, Lo, BRo, (uint32_t)nb[1] * (uint32_t)fp.Ls + (uint32_t)m.s, lds);
    force_dir<2>(fp, m, k, Lo, BRo, (uint32_t)nb[2] * (uint32_t)fp.Ls + (uint32_t)m.s, lds);
    force_dir<3>(fp, m, k, Lo, BRo, (uint32_t)nb[3] * (uint32_t)fp.Ls + (uint32_t)m.s, lds);
}

// Lie-algebra force per link: F = TA(U G^+), TA(M) = (M - M^+)/2 - tr(M - M^+)/6,
// so that for U -> e^{eps X} U (X in su(3)) dS/deps = Re tr(F X).
__global__ __launch_bounds__(256) void lie_force_kernel(int64_t nlinks, const double2 *U,
                                                        const double2 *G, double2 *F)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlinks) return;
    cx<double> u[9], g[9], m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        u[e] = {U[l * 9 + e].x, U[l * 9 + e].y};
        g[e] = {G[l * 9 + e].x, G[l * 9 + e].y};
    }
    // M = U G^+: M_ab = sum_c U_ac conj(G_bc)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            cx<double> acc = {0, 0};
#pragma unroll
            for (int c = 0; c < 3; ++c) acc = cjmadd(acc, g[b * 3 + c], u[a * 3 + c]);
            m[a * 3 + b] = acc;
        }
    // anti-Hermitian part, then its trace removed (the trace is imaginary)
    const double tr = (m[0].i + m[4].i + m[8].i) / 3.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cx<double> x = m[a * 3 + b], y = m[b * 3 + a];
            double re = 0.5 * (x.r - y.r), im = 0.5 * (x.i + y.i);
            if (a == b) im -= tr;
            F[l * 9 + a * 3 + b] = make_double2(re, im);
        }
}

}  // namespace

hipError_t launch_lie_force(int64_t nlinks, const void *U, const void *G, void *F, hipStream_t st)
{
    hipLaunchKernelGGL(lie_force_kernel, dim3((unsigned)((nlinks + 255) / 256)), dim3(256), 0, st, nlinks,
                       static_cast<const double2 *>(U), static_cast<const double2 *>(G),
                       static_cast<double2 *>(F));
    return hipGetLastError();
}

hipError_t launch_force(const Geometry &g, const OpCoeffs &c, int parity, const int32_t *nbr,
                        const void *Lp, const void *Rp, const void *Ln, const void *Rn,
                        void *grad, hipStream_t st, double scale, bool accumulate, double mu)
{
    ForceParams fp{};
    fp.scale = scale;
    fp.ef = std::exp(mu);
    fp.eb = std::exp(-mu);
    fp.accumulate = accumulate ? 1 : 0;
    fp.Lp = static_cast<const char *>(Lp);
    fp.Rp = static_cast<const char *>(Rp);
    fp.Ln = static_cast<const char *>(Ln);
    fp.Rn = static_cast<const char *>(Rn);
    fp.nbr = nbr + (int64_t)parity * 8 * g.Vh;
    fp.canon_of = g.canon_of + (int64_t)parity * g.Vh;
    fp.grad = static_cast<double2 *>(grad);
    fp.Vh = g.Vh;
    fp.N5 = g.N5;
    fp.V = g.V;
    fp.Ls = g.Ls;
    fp.spw = 64 / g.Ls;
    fp.c = c;
    const int64_t blocks = site_kernel_blocks(g);
    hipLaunchKernelGGL(force_kernel, dim3((unsigned)blocks), dim3(BLOCK), 0, st, fp);
    return hipGetLastError();
}


namespace {

constexpr int SQ_BLOCK = 256;

__global__ __launch_bounds__(SQ_BLOCK) void sumsq_partials_kernel(const double *x, int64_t n,
                                                                 double *partials)
{
    double v = 0;
    for (int64_t k = (int64_t)blockIdx.x * SQ_BLOCK + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * SQ_BLOCK)
        v += x[k] * x[k];
    __shared__ double red[SQ_BLOCK / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < SQ_BLOCK / 64; ++w) t += red[w];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(SQ_BLOCK) void sum_partials_kernel(const double *partials, int64_t n,
                                                               double *out)
{
    __shared__ double sm[SQ_BLOCK];
    double t = 0;
    for (int64_t k = threadIdx.x; k < n; k += SQ_BLOCK) t += partials[k];
    sm[threadIdx.x] = t;
    __syncthreads();
    for (int w = SQ_BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sm[0];
}

}  // namespace

int64_t norm2_blocks(int64_t n)
{
    const int64_t b = (n + SQ_BLOCK - 1) / SQ_BLOCK;
    return b < 2048 ? (b > 0 ? b : 1) : 2048;
}

hipError_t launch_norm2_f64(const double *x, int64_t n, double *partials, double *out, hipStream_t st)
{
    const int64_t nb = norm2_blocks(n);
    hipLaunchKernelGGL(sumsq_partials_kernel, dim3((unsigned)nb), dim3(SQ_BLOCK), 0, st, x, n, partials);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(SQ_BLOCK), 0, st, partials, nb, out);
    return hipGetLastError();
}

}  // namespace mobius
