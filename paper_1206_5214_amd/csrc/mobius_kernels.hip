// mobius_kernels.hip -- HIP kernels for gfx950 (MI355X) of the red/black
// Moebius domain-wall operator (Brower, Neff, Orginos, Sec. 3 and Sec. 4.1).
//
// Thread mapping of the site kernels: one lane per (4d site, s).  A 64-lane
// wavefront holds floor(64 / Ls) whole 4d sites, their Ls slices in
// consecutive lanes, so that
//  * every lane of a site reads the same eight links (one cache line serves
//    all Ls lanes: the links are read from HBM once per 4d site and reused
//    across the fifth dimension),
//  * the b5/c5 coupling between s-1, s, s+1 (the "vector gather" of Sec. 4.1)
//    is a cross-lane shuffle inside the wavefront,
//  * the Ls-direction solves I^-1 (closed-form elimination, Sec. 3) run in the
//    same wavefront through LDS, one lane per colour-spin component.
// Packed layouts are described in mobius_internal.h.
#include "mobius_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

namespace mobius {
namespace {

// ---------------------------------------------------------------------------
// hop kernel: out = epilogue( -1/2 sum_mu [...] )  on every s-slice


// PF: software pipelining of the direction loop.  0: operands of direction d
// are loaded in segment d; 1: the neighbour spinor of direction d+1 is loaded
// while direction d computes; 2: its link as well.  The eight neighbour
// indices are always loaded up front.
template <int P, bool DAG, int EPI, int PF>
__device__ __forceinline__ void hop_block(const HopParams &hp, int64_t lb)
{
    using S = Spin<P>;
    using T = typename S::T;
    const SiteMap m = site_map_lb(hp.Ls, hp.spw, hp.Vh, lb);
    const Coef<T> k = make_coef<T>(hp.c);
    const int Ls = hp.Ls;
    const uint32_t Vh = (uint32_t)hp.Vh, N5 = (uint32_t)hp.N5;
    const uint32_t i = (uint32_t)m.i;
    const uint32_t k5 = i * (uint32_t)Ls + (uint32_t)m.s;
    const int64_t fbytes = S::bytes(hp.N5);
    const Buf blink(hp.links, (int64_t)8 * hp.Vh * Link<P>::REC);
    const Buf bnbr(hp.nbr, 8 * hp.Vh * 4);

    if (hp.active) {  // a system group whose systems have all converged: nothing to stage
        bool any = false;
        for (int r = 0; r < hp.nrhs; ++r) any = any || hp.active[r];
        if (!any) return;
    }

    extern __shared__ u32x4 dyn_lds[];
    LinkSource<P> ls;
    ls.glob = &blink;
    ls.lds = nullptr;
    ls.Vh = Vh;
    ls.i = i;
    ls.sites_blk = (uint32_t)(WAVES * hp.spw);
    // lanes without a site (idle tail lanes of a wavefront) read record 0
    ls.sib = m.site_ok ? (uint32_t)(m.wave * hp.spw + m.g) : 0u;
    if (hp.stage_links && P == MOBIUS_F16) {
        // one thread per (direction, site): the record expanded to the dot2 operand form
        constexpr uint32_t REC = Link<P>::REC;
        const uint32_t i0 = (uint32_t)(lb * WAVES * hp.spw);
        const uint32_t nsites = min(ls.sites_blk, Vh - i0);
        for (uint32_t c = threadIdx.x; c < 8u * nsites; c += BLOCK) {
            const uint32_t d = c / nsites, j = c - d * nsites;
            u32x4 q[3];
#pragma unroll
            for (int w = 0; w < 3; ++w)
                q[w] = hp.nt ? blink.ld16_nt((i0 + j) * REC + 16u * w, d * Vh * REC)
                             : blink.ld16((i0 + j) * REC + 16u * w, d * Vh * REC);
            half2v u[9];
            Link<MOBIUS_F16>::raw_from_words(q, u);
            constexpr uint32_t W = (PF == 3 ? LINKROW_REC : LINKH2_REC) / 16;
            u32x4 *dst = dyn_lds + (size_t)(d * ls.sites_blk + j) * W;
            if (d < 4)
                stage_link_f16<true, PF == 3>(u, dst);
            else
                stage_link_f16<false, PF == 3>(u, dst);
        }
        ls.lds = reinterpret_cast<const char *>(dyn_lds);
    } else if (hp.stage_links) {
        constexpr uint32_t REC = Link<P>::REC;
        const uint32_t i0 = (uint32_t)(lb * WAVES * hp.spw);
        const uint32_t nsites = min(ls.sites_blk, Vh - i0);
        const uint32_t cpd = nsites * REC / 16u;  // 16-byte words per direction
        for (uint32_t c = threadIdx.x; c < 8u * cpd; c += BLOCK) {
            const uint32_t d = c / cpd, q = c - d * cpd;
            const u32x4 v = hp.nt ? blink.ld16_nt(i0 * REC + q * 16u, d * Vh * REC)
                                  : blink.ld16(i0 * REC + q * 16u, d * Vh * REC);
            dyn_lds[(d * ls.sites_blk * REC) / 16u + q] = v;
        }
        ls.lds = reinterpret_cast<const char *>(dyn_lds);
    }

    uint32_t jn[8];
    {
        const u32x4 n0 = bnbr.ld16(i * 32u, 0u), n1 = bnbr.ld16(i * 32u + 16u, 0u);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            jn[d] = n0[d] * (uint32_t)Ls + (uint32_t)m.s;
            jn[4 + d] = n1[d] * (uint32_t)Ls + (uint32_t)m.s;
        }
    }

    if (hp.stage_links) __syncthreads();

    for (int r = 0; r < hp.nrhs; ++r) {
    if (hp.active && !hp.active[r]) continue;
    const Buf bin(hp.in + r * hp.fstride, fbytes), bout(hp.out + r * hp.fstride, fbytes);
    const char *xr = hp.x ? hp.x + r * hp.fstride : nullptr;
    const char *yr = hp.y ? hp.y + r * hp.fstride : nullptr;

    cx<T> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
    // B = b5 + c5 C5 applied to the neighbours here (forward hop), unless the
    // input already holds B in (written so by an EPI_BMIX epilogue)
    constexpr bool MIXIN = !DAG && (EPI & EPI_PREMIXED) == 0;

    // B weights of this lane (per-slice b5(s), c5(s) when the operator has them)
    const MixW<T> wB = mix_w(k, false, m, Ls, false);
    if constexpr (P == MOBIUS_F16) {
        // forward block: B mixing weights of this lane (norms folded in per direction)
        const float wu = MIXIN ? (float)wB.bu * (m.s == 0 ? -(float)k.mf : 1.f) : 0.f;
        const float wl = MIXIN ? (float)wB.bl * (m.s == Ls - 1 ? -(float)k.mf : 1.f) : 0.f;
        // PF 3: the colour multiply on the matrix cores, links and neighbour
        // spinors prefetched one direction ahead
        constexpr bool MF = PF == 3;
        const int quad = m.lane & 3;
        // (its spinors two directions ahead: the registers the colour
        // multiply frees hold one more direction in flight)
        RawH nx, nx2;
        LinkH2 unx;
        LinkRows rnx;
        load_raw_f16(bin, N5, jn[0], nx);
        if constexpr (MF) {
            load_raw_f16(bin, N5, jn[1], nx2);
            ls.get_rows(0, quad, rnx);
        } else if constexpr (PF >= 2) {
            ls.template get_h2<true>(0, unx);
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const RawH o = nx;
            if constexpr (MF) {
                nx = nx2;
                if (d < 6) load_raw_f16(bin, N5, jn[d + 2], nx2);
            } else {
                if (d < 7) load_raw_f16(bin, N5, jn[d + 1], nx);
            }
            LinkH2 u;
            LinkRows ur;
            if constexpr (MF) {
                ur = rnx;
                if (d < 7) ls.get_rows(d + 1, quad, rnx);
            } else if constexpr (PF >= 2) {
                u = unx;
                if (d < 3)
                    ls.template get_h2<true>(d + 1, unx);
                else if (d < 7)
                    ls.template get_h2<false>(d + 1, unx);
            } else {
                if (d < 4)
                    ls.template get_h2<true>(d, u);
                else
                    ls.template get_h2<false>(d, u);
            }
            constexpr int SF = DAG ? +1 : -1;
            const int sig = d < 4 ? SF : -SF;
            half2v um[6], lp[6];
            float al, bu = 0.f, bl = 0.f;
            if constexpr (MIXIN) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    um[c] = shfl_h2(o.c[c], m.lm);
                    lp[c] = shfl_h2(o.c[6 + c], m.lp);
                }
                al = (float)wB.a * o.n;
                bu = wu * __shfl(o.n, m.lm, 64);
                bl = wl * __shfl(o.n, m.lp, 64);
            } else {
                al = o.n;
            }
            (void)sig;
            // weights divided by the largest of them (the binary16 step keeps
            // every term O(1)); the scale is restored in FP32
            const float sc = fmaxf(fabsf(al), fmaxf(fabsf(bu), fabsf(bl)));
            // (hardware reciprocal: its last-bit error scales both the
            // binary16 terms and their restoration, so it cancels)
            const float inv = sc > 0.f ? __builtin_amdgcn_rcpf(sc) : 0.f;
            const half2v al2 = splat_h2(al * inv), bu2 = splat_h2(bu * inv), bl2 = splat_h2(bl * inv);
            half2v hh[6];
#define MOBIUS_HS(MU, SG) half_spinor_h2<MU, SG, MIXIN>(o.c, um, lp, al2, bu2, bl2, hh)
#define MOBIUS_LA(MU, SG)                                                                          \
    if constexpr (MF)                                                                              \
        link_accumulate_mfma<MU, SG>(hh, -0.5f * sc, ur, acc);                                     \
    else                                                                                           \
        link_accumulate_h2<MU, SG>(hh, -0.5f * sc, u, acc)
            switch (d) {
            case 0: MOBIUS_HS(0, SF); MOBIUS_LA(0, SF); break;
            case 1: MOBIUS_HS(1, SF); MOBIUS_LA(1, SF); break;
            case 2: MOBIUS_HS(2, SF); MOBIUS_LA(2, SF); break;
            case 3: MOBIUS_HS(3, SF); MOBIUS_LA(3, SF); break;
            case 4: MOBIUS_HS(0, -SF); MOBIUS_LA(0, -SF); break;
            case 5: MOBIUS_HS(1, -SF); MOBIUS_LA(1, -SF); break;
            case 6: MOBIUS_HS(2, -SF); MOBIUS_LA(2, -SF); break;
            default: MOBIUS_HS(3, -SF); MOBIUS_LA(3, -SF); break;
            }
#undef MOBIUS_LA
#undef MOBIUS_HS
#pragma unroll
            for (int c = 0; c < 12; ++c) pin(acc[c]);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
    cx<T> nxt[12], unx[9];
    if constexpr (PF >= 1) S::load(bin, N5, jn[0], nxt);
    if constexpr (PF >= 2) ls.get(0, unx);

#pragma unroll
    for (int d = 0; d < 8; ++d) {
        cx<T> chi[12], u[9];
        if constexpr (PF >= 1) {
#pragma unroll
            for (int c = 0; c < 12; ++c) chi[c] = nxt[c];
            if (d < 7) S::load(bin, N5, jn[d + 1], nxt);
        } else {
            S::load(bin, N5, jn[d], chi);
        }
        if constexpr (PF >= 2) {
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = unx[e];
            if (d < 7) ls.get(d + 1, unx);
        } else {
            ls.get(d, u);
        }
        if constexpr (MIXIN) {
            // B = b5 + c5 C5 on the input: gather s-1, s, s+1 of the neighbour
            mix_s(chi, wB, k.mf, m, Ls, false);
        }
        constexpr int SF = DAG ? +1 : -1;  // forward projector (1 -+ g_mu)
        switch (d) {
        case 0: hop_dir<P, 0, true, SF>(chi, u, acc); break;
        case 1: hop_dir<P, 1, true, SF>(chi, u, acc); break;
        case 2: hop_dir<P, 2, true, SF>(chi, u, acc); break;
        case 3: hop_dir<P, 3, true, SF>(chi, u, acc); break;
        case 4: hop_dir<P, 0, false, -SF>(chi, u, acc); break;
        case 5: hop_dir<P, 1, false, -SF>(chi, u, acc); break;
        case 6: hop_dir<P, 2, false, -SF>(chi, u, acc); break;
        default: hop_dir<P, 3, false, -SF>(chi, u, acc); break;
        }
        // the accumulator is complete here; nothing of direction d+1 beyond
        // its prefetched loads moves above this point
#pragma unroll
        for (int c = 0; c < 12; ++c) pin(acc[c]);
        __builtin_amdgcn_sched_barrier(0);
    }
    }
    // the -1/2 of the hopping term (the FP16 loop folds it into each
    // direction's scale, a power of two, so the result is the same)
    if constexpr (P != MOBIUS_F16) {
        const T mhalf = (T)-0.5;
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = mhalf * acc[c];
    }

    {
    // coefficients of the epilogue, converted here so that none of them is
    // held in a register across the direction loop
    const Coef<T> k = make_coef<T>(hp.c);
    if constexpr (DAG && (EPI & EPI_NOBOUT) == 0) {  // B^+ on the output
        if (!k.ls)
            mix_s(acc, k.b5, k.c5, k.mf, m, Ls, true);
        else
            mix_s(acc, mix_w(k, false, m, Ls, true), k.mf, m, Ls, true);
    }
    if constexpr ((EPI & EPI_M5ADD) != 0) {
        cx<T> yv[12];
        S::load(Buf(yr, fbytes), N5, k5, yv);
        mix_s(yv, mix_w(k, true, m, Ls, DAG), k.mf, m, Ls, DAG);  // I y = M+ y + M- C5 y
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] + yv[c];
    }
    if constexpr ((EPI & EPI_M5SUB) != 0) {
        cx<T> yv[12];
        S::load(Buf(yr, fbytes), N5, k5, yv);
        mix_s(yv, mix_w(k, true, m, Ls, DAG), k.mf, m, Ls, DAG);  // I y (I^+ y)
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = yv[c] - acc[c];
    }
    if constexpr ((EPI & EPI_PRESUB) != 0) {
        cx<T> xv[12];
        S::load(Buf(xr, fbytes), N5, k5, xv);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = xv[c] - acc[c];
    }
    if constexpr ((EPI & EPI_M5INV) != 0) {
        // the buffer lives in the dynamic LDS; where it overlays the staged
        // links, every wave of the block must be past its direction loop
        if (hp.m5_off == 0 && hp.stage_links) __syncthreads();
        M5Lds<T> &lds = *reinterpret_cast<M5Lds<T> *>(reinterpret_cast<char *>(dyn_lds) + hp.m5_off);
        m5inv_lanes(acc, k, m, Ls, DAG, lds);
    }
    if constexpr ((EPI & EPI_BMIX) != 0)  // B r (B^+ r in the adjoint hop)
        mix_s(acc, mix_w(k, false, m, Ls, DAG), k.mf, m, Ls, DAG);
    if constexpr ((EPI & EPI_POSTSUB) != 0) {
        cx<T> xv[12];
        S::load(Buf(xr, fbytes), N5, k5, xv);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = xv[c] - acc[c];
    }
    if constexpr ((EPI & EPI_NORM) != 0) {
        // |stored value|^2, from the encoded registers
        double n = 0;
        if (m.site_ok) n = S::store_norm2(bout, N5, k5, acc);
        block_sum_store(n, hp.partials + r * hp.pstride, lb);
    } else {
        if (m.site_ok) S::store(bout, N5, k5, acc);
    }
    }
    }  // rhs
}

// The binary16 matrix-core loop is held to 128 VGPRs (four waves per SIMD):
// its adjoint hop with the I^-+ epilogue needs 130 on its own and then runs
// three waves (the cap costs it one spilled dword pair; the FP16 solve runs
// about 1 % faster).  The FP64 hop spills heavily under a three-wave cap and
// keeps two.
template <int P, bool DAG, int EPI, int PF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(P == MOBIUS_F16 && PF == 3 ? 4 : 1)))
void hop_kernel(HopParams hp)
{
    hop_block<P, DAG, EPI, PF>(hp, logical_block(hp.remap));
}

// Persistent launch over a batch of lattices of uneven size: a fixed grid
// walks the concatenated block lists of all groups (group j owns work items
// [prefix[j], prefix[j+1])); every workgroup exits after its last item.
template <int P, bool DAG, int EPI, int PF>
__global__ __launch_bounds__(BLOCK) void hop_batch_kernel(const HopParams *groups, int ngroups,
                                                          const int64_t *prefix)
{
    const int64_t total = prefix[ngroups];
    int j = 0;
    // XCD-contiguous order (as the single-lattice launch with remap on) over
    // the n = min(grid, items) workgroups that have work, so that every XCD
    // takes an eighth of the items and each its own contiguous range
    const int64_t n = total < (int64_t)gridDim.x ? total : (int64_t)gridDim.x;
    const int64_t b = blockIdx.x;
    if (b >= n) return;
    const int64_t q = n / NUM_XCD, rem = n % NUM_XCD, x = b % NUM_XCD;
    for (int64_t w = x * q + (x < rem ? x : rem) + b / NUM_XCD; w < total; w += n) {
        while (w >= prefix[j + 1]) ++j;
        hop_block<P, DAG, EPI, PF>(groups[j], w - prefix[j]);
        __syncthreads();  // LDS of this item is dead before the next item stages
    }
}

// per-site s-direction operators: kind 0 -> I (or I^+), kind 1 -> I^-1 (or I^-+)
template <int P, bool DAG, int KIND>
__global__ __launch_bounds__(BLOCK) void m5_kernel(const char *in, char *out, int64_t Vh,
                                                   int64_t N5, int Ls, int spw, OpCoeffs c)
{
    using S = Spin<P>;
    using T = typename S::T;
    const SiteMap m = site_map(Ls, spw, Vh);
    const Coef<T> k = make_coef<T>(c);
    const uint32_t k5 = (uint32_t)m.i * (uint32_t)Ls + (uint32_t)m.s;
    const int64_t fbytes = S::bytes(N5);
    cx<T> v[12];
    S::load(Buf(in, fbytes), (uint32_t)N5, k5, v);
    if constexpr (KIND == 0) {
        mix_s(v, mix_w(k, true, m, Ls, DAG), k.mf, m, Ls, DAG);
    } else {
        __shared__ M5Lds<T> lds;
        m5inv_lanes(v, k, m, Ls, DAG, lds);
    }
    if (m.site_ok) S::store(Buf(out, fbytes), (uint32_t)N5, k5, v);
}

// ---------------------------------------------------------------------------
// geometry, packing

__device__ __forceinline__ void coords_of(int64_t c, const int *L, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(c % L[mu]);
        c /= L[mu];
    }
}

__device__ __forceinline__ int64_t canon_index(const int x[4], const int *L)
{
    return (((int64_t)x[3] * L[2] + x[2]) * L[1] + x[1]) * L[0] + x[0];
}

struct Dims {
    int L[4];
};

// nbr[p][i][d] = packed index of the d-th neighbour of packed site i of parity p
__global__ void build_nbr_kernel(Dims D, int64_t Vh, const int32_t *canon_of,
                                 const int32_t *packed_of, int32_t *nbr)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * Vh) return;
    const int64_t c = canon_of[t];
    int x[4];
    coords_of(c, D.L, x);
    for (int d = 0; d < 8; ++d) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        const int mu = d & 3;
        const int dir = d < 4 ? 1 : -1;
        y[mu] = (y[mu] + dir + D.L[mu]) % D.L[mu];
        nbr[t * 8 + d] = packed_of[canon_index(y, D.L)];
    }
}

template <int P>
__device__ __forceinline__ void put_link_elem(char *dst, int64_t idx, double re, double im)
{
    if constexpr (P == MOBIUS_F64) {
        reinterpret_cast<double2 *>(dst)[idx] = make_double2(re, im);
    } else if constexpr (P == MOBIUS_F32) {
        reinterpret_cast<float2 *>(dst)[idx] = make_float2((float)re, (float)im);
    } else {
        half2v h;
        h.x = (_Float16)re;
        h.y = (_Float16)im;
        reinterpret_cast<half2v *>(dst)[idx] = h;
    }
}

// record (p, d, i) of the packed links; padding elements are zero
template <int P>
// sf, sb: factors of the time-like forward (d = 3) and backward (d = 7)
// records (e^{+-mu} of a chemical potential; 1 without one)
__global__ void pack_links_kernel(Dims D, int64_t V, int64_t Vh, const int32_t *canon_of,
                                  const double2 *canon, char *packed, double sf, double sb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * Vh * 8) return;
    const int64_t i = t % Vh;
    const int d = (int)((t / Vh) % 8);
    const int p = (int)(t / (Vh * 8));
    const int64_t c = canon_of[p * Vh + i];
    int x[4];
    coords_of(c, D.L, x);
    const int mu = d & 3;
    if (d >= 4) x[mu] = (x[mu] - 1 + D.L[mu]) % D.L[mu];
    const int64_t src = ((int64_t)mu * V + canon_index(x, D.L)) * 9;
    constexpr int REC = Link<P>::REC;
    constexpr int EB = P == MOBIUS_F64 ? 16 : P == MOBIUS_F32 ? 8 : 4;
    char *rec = packed + (((int64_t)p * 8 + d) * Vh + i) * REC;
    const double f = d == 3 ? sf : d == 7 ? sb : 1.0;
    for (int e = 0; e < REC / EB; ++e) {
        double2 u = e < 9 ? canon[src + e] : make_double2(0.0, 0.0);
        put_link_elem<P>(rec, e, f * u.x, f * u.y);
    }
}

// Walls of the fifth dimension (Sec. 2.2): the chiral shift P_{ss'} =
// delta_{ss'} P- + delta_{s',s+1 mod Ls} P+ puts a 4d field b on slice 0 as
// P- b and on slice Ls-1 as P+ b, and q = (P^+ psi)_0 = P- psi_0 + P+ psi_{Ls-1}
// reads one back.  Canonical layouts, P+ = spins 0, 1 (components 0..5).
__global__ __launch_bounds__(256) void wall_place_kernel(int64_t V, int Ls, int64_t n,
                                                         const double2 *b4, double2 *eta5)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (rhs, s, x)
    if (t >= n) return;
    const int64_t x = t % V, rs = t / V;
    const int s = (int)(rs % Ls);
    const int64_t r = rs / Ls;
    const double2 *src = b4 + (r * V + x) * 12;
    double2 *dst = eta5 + t * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const bool take = q < 6 ? s == Ls - 1 : s == 0;
        dst[q] = take ? src[q] : make_double2(0.0, 0.0);
    }
}

__global__ __launch_bounds__(256) void wall_read_kernel(int64_t V, int Ls, int64_t n,
                                                        const double2 *psi5, double2 *q4)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (rhs, x)
    if (t >= n) return;
    const int64_t x = t % V, r = t / V;
    const double2 *lo = psi5 + ((r * Ls + 0) * V + x) * 12;
    const double2 *hi = psi5 + ((r * Ls + Ls - 1) * V + x) * 12;
    double2 *dst = q4 + t * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) dst[q] = q < 6 ? hi[q] : lo[q];
}

// Bulk reconstruction from the overlap solution (Sec. 2.3): with y the
// Pauli-Villars solution D_DW(1) y = D_DW(m) P psi~,  Omega = P^+ y,
// (P^+ y)_s = P- y_s + P+ y_{s-1 mod Ls}, and Psi_0 = psi, Psi_s = -Omega_s.
__global__ __launch_bounds__(256) void bulk_assemble_kernel(int64_t V, int Ls, int64_t n,
                                                            const double2 *psi4, const double2 *y5,
                                                            double2 *Psi5)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (rhs, s, x)
    if (t >= n) return;
    const int64_t x = t % V, rs = t / V;
    const int s = (int)(rs % Ls);
    const int64_t r = rs / Ls;
    double2 *dst = Psi5 + t * 12;
    if (s == 0) {
        const double2 *src = psi4 + (r * V + x) * 12;
#pragma unroll
        for (int q = 0; q < 12; ++q) dst[q] = src[q];
        return;
    }
    const double2 *ys = y5 + t * 12, *ym = y5 + ((r * Ls + s - 1) * V + x) * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const double2 v = q < 6 ? ym[q] : ys[q];  // P+ from s-1, P- from s
        dst[q] = make_double2(-v.x, -v.y);
    }
}

// canonical [s][t][z][y][x][12] complex128 <-> packed halves
template <int P>
__global__ __launch_bounds__(256) void pack_spinor_kernel(int64_t Vh, int Ls,
                                                          const int32_t *canon_of,
                                                          const double2 *canon, char *even,
                                                          char *odd)
{
    using S = Spin<P>;
    using T = typename S::T;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N5 = Vh * Ls;
    if (t >= 2 * N5) return;
    const int p = (int)(t / N5);
    const int64_t k5 = t - p * N5;
    const int64_t i = k5 / Ls;
    const int s = (int)(k5 - i * Ls);
    const int64_t V = 2 * Vh;
    const int64_t c = canon_of[p * Vh + i];
    const double2 *src = canon + ((int64_t)s * V + c) * 12;
    cx<T> v[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        double2 z = src[q];
        v[q] = {(T)z.x, (T)z.y};
    }
    S::store(Buf(p == 0 ? even : odd, S::bytes(N5)), (uint32_t)N5, (uint32_t)k5, v);
}

template <int P>
__global__ __launch_bounds__(256) void unpack_spinor_kernel(int64_t Vh, int Ls,
                                                            const int32_t *canon_of,
                                                            const char *even, const char *odd,
                                                            double2 *canon)
{
    using S = Spin<P>;
    using T = typename S::T;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N5 = Vh * Ls;
    if (t >= 2 * N5) return;
    const int p = (int)(t / N5);
    const int64_t k5 = t - p * N5;
    const int64_t i = k5 / Ls;
    const int s = (int)(k5 - i * Ls);
    const int64_t V = 2 * Vh;
    const int64_t c = canon_of[p * Vh + i];
    cx<T> v[12];
    S::load(Buf(p == 0 ? even : odd, S::bytes(N5)), (uint32_t)N5, (uint32_t)k5, v);
    double2 *dst = canon + ((int64_t)s * V + c) * 12;
#pragma unroll
    for (int q = 0; q < 12; ++q) dst[q] = make_double2((double)v[q].r, (double)v[q].i);
}

// ---------------------------------------------------------------------------
// BLAS-1 and reductions (one thread per site5)

constexpr int BLAS_BLOCK = 256;

// A packed field of `n5` 5d sites filled with seeded pseudo-random values in
// [-1, 1) (FP16: binary16 components with site norms in [1, 2)), from a
// 32-bit hash of the word index: launch-parameter timing on data with the
// magnitudes of a Gaussian field rather than on zeros.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int P>
__global__ void fill_random_kernel(char *out, int64_t n5, uint32_t seed)
{
    const int64_t words = Spin<P>::bytes(n5) / 4;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = mix32((uint32_t)w * 2654435761u ^ seed);
        const float u = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;  // [-1, 1)
        uint32_t v;
        if constexpr (P == MOBIUS_F64) {
            // the high word of a double in [-1, 1) with this word's low 32 bits
            const double d = (double)u;
            const uint64_t b = __builtin_bit_cast(uint64_t, d);
            v = (w & 1) ? (uint32_t)(b >> 32) : h;
        } else if constexpr (P == MOBIUS_F32) {
            v = __builtin_bit_cast(uint32_t, u);
        } else {
            if (w >= 3 * 4 * n5) {  // the site norms
                v = __builtin_bit_cast(uint32_t, 1.5f + 0.5f * u);
            } else {
                const _Float16 a = (_Float16)u, b = (_Float16)(-0.5f * u);
                v = (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
            }
        }
        reinterpret_cast<uint32_t *>(out)[w] = v;
    }
}

__global__ void zero_kernel(uint4 *p, int64_t n16, unsigned char *tail, int64_t ntail)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) p[k] = make_uint4(0, 0, 0, 0);
    if (k < ntail) tail[k] = 0;
}

// ---------------------------------------------------------------------------
// batched vector kernels: blockIdx.y selects the system (one lattice and one
// right-hand side); systems whose active flag is zero return at once.

__device__ __forceinline__ bool sys_inactive(const VecSys &v, const int32_t *active)
{
    return v.flag >= 0 && active && active[v.flag] == 0;
}

// x (PX) += alpha p;  r -= alpha q;  partials of |r|^2.  a = x, b = p, c = r, d = q, s0 = alpha
// (a null: r and its norm only, x is updated elsewhere).
template <int P, int PX>
__global__ __launch_bounds__(BLAS_BLOCK) void cg_xr_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using SX = Spin<PX>;
    using T = typename S::T;
    using TX = typename SX::T;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if ((int64_t)blockIdx.x * BLAS_BLOCK >= v.N5) return;
    double n = 0;
    if (k < v.N5) {
        const T al = (T)*v.s0;
        const TX alx = (TX)*v.s0;
        const int64_t fb = S::bytes(v.N5);
        const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
        const Buf bx(v.a, SX::bytes(v.N5)), bp(v.b, fb), br(v.c, fb), bq(v.d, fb);
        cx<TX> xv[12];
        cx<T> pv[12], rv[12];
        if (v.a) {
            SX::load(bx, n5, kk, xv);
            S::load(bp, n5, kk, pv);
#pragma unroll
            for (int c = 0; c < 12; ++c) xv[c] = xv[c] + alx * cx<TX>{(TX)pv[c].r, (TX)pv[c].i};
            SX::store(bx, n5, kk, xv);
        }
        S::load(br, n5, kk, rv);
        S::load(bq, n5, kk, pv);
#pragma unroll
        for (int c = 0; c < 12; ++c) rv[c] = rv[c] - al * pv[c];
        n = S::store_norm2(br, n5, kk, rv);
    }
    block_sum_store(n, v.partials, blockIdx.x);
}

// d = s0 * a + s1 * b  (null scalar = 1); optional partials of |d|^2
template <int P, bool NORM>
__global__ __launch_bounds__(BLAS_BLOCK) void axpby_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using T = typename S::T;
    if ((int64_t)blockIdx.x * BLAS_BLOCK >= v.N5) return;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double n = 0;
    if (k < v.N5) {
        const T av = v.s0 ? (T)*v.s0 : (T)1, bv = v.s1 ? (T)*v.s1 : (T)1;
        const int64_t fb = S::bytes(v.N5);
        const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
        cx<T> xv[12], yv[12];
        S::load(Buf(v.a, fb), n5, kk, xv);
        S::load(Buf(v.b, fb), n5, kk, yv);
#pragma unroll
        for (int c = 0; c < 12; ++c) xv[c] = av * xv[c] + bv * yv[c];
        if constexpr (NORM)
            n = S::store_norm2(Buf(v.d, fb), n5, kk, xv);
        else
            S::store(Buf(v.d, fb), n5, kk, xv);
    }
    if constexpr (NORM) block_sum_store(n, v.partials, blockIdx.x);
}

// partials of |a|^2
template <int P>
__global__ __launch_bounds__(BLAS_BLOCK) void norm2_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using T = typename S::T;
    if ((int64_t)blockIdx.x * BLAS_BLOCK >= v.N5) return;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double n = 0;
    if (k < v.N5) {
        cx<T> x[12];
        S::load(Buf(v.a, S::bytes(v.N5)), (uint32_t)v.N5, (uint32_t)k, x);
        n = site_norm2(x);
    }
    block_sum_store(n, v.partials, blockIdx.x);
}

// precision conversion b (PO) = a (PI); accumulate: d (F64) += a (PI)
template <int PI, int PO>
__global__ __launch_bounds__(BLAS_BLOCK) void convert_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    cx<typename Spin<PI>::T> x[12];
    Spin<PI>::load(Buf(v.a, Spin<PI>::bytes(v.N5)), (uint32_t)v.N5, (uint32_t)k, x);
    cx<typename Spin<PO>::T> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(typename Spin<PO>::T)x[c].r, (typename Spin<PO>::T)x[c].i};
    Spin<PO>::store(Buf(v.b, Spin<PO>::bytes(v.N5)), (uint32_t)v.N5, (uint32_t)k, w);
}

template <int PI>
__global__ __launch_bounds__(BLAS_BLOCK) void accumulate_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    cx<typename Spin<PI>::T> x[12];
    Spin<PI>::load(Buf(v.a, Spin<PI>::bytes(v.N5)), (uint32_t)v.N5, (uint32_t)k, x);
    cx<double> h[12];
    const Buf bh(v.d, Spin<MOBIUS_F64>::bytes(v.N5));
    Spin<MOBIUS_F64>::load(bh, (uint32_t)v.N5, (uint32_t)k, h);
#pragma unroll
    for (int c = 0; c < 12; ++c) h[c] = {h[c].r + (double)x[c].r, h[c].i + (double)x[c].i};
    Spin<MOBIUS_F64>::store(bh, (uint32_t)v.N5, (uint32_t)k, h);
    // the low-precision correction is consumed: clear it
    cx<typename Spin<PI>::T> z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = {0, 0};
    Spin<PI>::store(Buf(v.a, Spin<PI>::bytes(v.N5)), (uint32_t)v.N5, (uint32_t)k, z);
}

// x (PX) += alpha p_old;  p = s + beta p_old.  a = s, b = p, c = x, s0 = alpha, s1 = beta.
// (The x update of a CG step moved here from the r update: p_old is read anyway.)
template <int P, int PX>
__global__ __launch_bounds__(BLAS_BLOCK) void pupd_x_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using SX = Spin<PX>;
    using T = typename S::T;
    using TX = typename SX::T;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    const TX al = (TX)*v.s0;
    const T be = (T)*v.s1;
    const int64_t fb = S::bytes(v.N5);
    const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
    const Buf bs(v.a, fb), bp(v.b, fb), bx(v.c, SX::bytes(v.N5));
    cx<T> sv[12], pv[12];
    cx<TX> xv[12];
    S::load(bp, n5, kk, pv);
    SX::load(bx, n5, kk, xv);
#pragma unroll
    for (int c = 0; c < 12; ++c) xv[c] = xv[c] + al * cx<TX>{(TX)pv[c].r, (TX)pv[c].i};
    SX::store(bx, n5, kk, xv);
    S::load(bs, n5, kk, sv);
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = sv[c] + be * pv[c];
    S::store(bp, n5, kk, pv);
}

// x (PX) += alpha p.  a = p, c = x, s0 = alpha.
template <int P, int PX>
__global__ __launch_bounds__(BLAS_BLOCK) void xflush_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using SX = Spin<PX>;
    using TX = typename SX::T;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    const TX al = (TX)*v.s0;
    const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
    const Buf bx(v.c, SX::bytes(v.N5));
    cx<typename S::T> pv[12];
    cx<TX> xv[12];
    S::load(Buf(v.a, S::bytes(v.N5)), n5, kk, pv);
    SX::load(bx, n5, kk, xv);
#pragma unroll
    for (int c = 0; c < 12; ++c) xv[c] = xv[c] + al * cx<TX>{(TX)pv[c].r, (TX)pv[c].i};
    SX::store(bx, n5, kk, xv);
}

// p[slot] = s + beta p[prev] in a ring of directions (the deferred x update
// keeps one chunk's directions).  a = s, b = p[0], slots sstride bytes apart,
// s1 = beta.
template <int P>
__global__ __launch_bounds__(BLAS_BLOCK) void pupd_ring_batch(const VecSys *sys, const int32_t *active,
                                                              int slot, int prev)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using T = typename S::T;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    const T be = (T)*v.s1;
    const int64_t fb = S::bytes(v.N5);
    const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
    cx<T> sv[12], pv[12];
    S::load(Buf(v.b + prev * v.sstride, fb), n5, kk, pv);
    S::load(Buf(v.a, fb), n5, kk, sv);
#pragma unroll
    for (int c = 0; c < 12; ++c) pv[c] = sv[c] + be * pv[c];
    S::store(Buf(v.b + slot * v.sstride, fb), n5, kk, pv);
}

// x (PX) += sum_{i < n} alpha_i p[i]: the x update of a chunk in one pass.
// b = p[0], slots sstride bytes apart, s0 = the alphas, c = x.
template <int P, int PX>
__global__ __launch_bounds__(BLAS_BLOCK) void xring_batch(const VecSys *sys, const int32_t *active, int n)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using SX = Spin<PX>;
    using TX = typename SX::T;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (k >= v.N5) return;
    const int64_t fb = S::bytes(v.N5);
    const uint32_t n5 = (uint32_t)v.N5, kk = (uint32_t)k;
    cx<TX> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cx<TX>{0, 0};
#pragma unroll 2
    for (int i = 0; i < n; ++i) {
        const TX al = (TX)v.s0[i];
        cx<typename S::T> pv[12];
        S::load(Buf(v.b + i * v.sstride, fb), n5, kk, pv);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] + al * cx<TX>{(TX)pv[c].r, (TX)pv[c].i};
    }
    const Buf bx(v.c, SX::bytes(v.N5));
    cx<TX> xv[12];
    SX::load(bx, n5, kk, xv);
#pragma unroll
    for (int c = 0; c < 12; ++c) xv[c] = xv[c] + acc[c];
    SX::store(bx, n5, kk, xv);
}

// r -= alpha q, |r|^2 per site block, and u = I^-+ r of the stored r, in the
// site-lane mapping of the hop so that the Ls-direction solve stays inside a
// wavefront.  a = r, b = q, c = u, s0 = alpha; one workgroup per site block.
template <int P>
__global__ __launch_bounds__(BLOCK) void rupd_m5inv_batch(const VecSys *sys, const int32_t *active,
                                                          int mode)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    const int Ls = v.Ls, spw = 64 / Ls;
    const int64_t Vh = v.N5 / Ls;
    const int64_t per_block = (int64_t)spw * WAVES;
    if ((int64_t)blockIdx.x * per_block >= Vh) return;  // uniform in the workgroup
    using S = Spin<P>;
    using T = typename S::T;
    const SiteMap m = site_map_lb(Ls, spw, Vh, blockIdx.x);
    const Coef<T> k = make_coef<T>(*v.coef);
    const uint32_t n5 = (uint32_t)v.N5, k5 = (uint32_t)m.i * (uint32_t)Ls + (uint32_t)m.s;
    const int64_t fb = S::bytes(v.N5);
    const Buf br(v.a, fb);
    cx<T> rv[12], qv[12];
    S::load(br, n5, k5, rv);
    S::load(Buf(v.b, fb), n5, k5, qv);
    const T al = (T)*v.s0;
#pragma unroll
    for (int c = 0; c < 12; ++c) rv[c] = rv[c] - al * qv[c];
    double n = 0;
    if (m.site_ok) n = S::store_norm2_q(br, n5, k5, rv);
    vmem_drain();
    block_sum_store(n, v.partials, blockIdx.x);
    if (mode == 2) return;  // uniform: no solve of the updated residual
    __shared__ M5Lds<T> lds;
    m5inv_lanes(rv, k, m, Ls, mode != 1, lds);
    if (mode == 3) mix_s(rv, k.b5, k.c5, k.mf, m, Ls, true);  // B^+ I^-+ r (left form)
    if (m.site_ok) S::store(Buf(v.c, fb), n5, k5, rv);
}

// partials of Re <a, b>
template <int P>
__global__ __launch_bounds__(BLAS_BLOCK) void dot_batch(const VecSys *sys, const int32_t *active)
{
    const VecSys v = sys[blockIdx.y];
    if (sys_inactive(v, active)) return;
    using S = Spin<P>;
    using T = typename S::T;
    if ((int64_t)blockIdx.x * BLAS_BLOCK >= v.N5) return;
    const int64_t k = (int64_t)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double n = 0;
    if (k < v.N5) {
        const int64_t fb = S::bytes(v.N5);
        cx<T> x[12], y[12];
        S::load(Buf(v.a, fb), (uint32_t)v.N5, (uint32_t)k, x);
        S::load(Buf(v.b, fb), (uint32_t)v.N5, (uint32_t)k, y);
#pragma unroll
        for (int c = 0; c < 12; ++c) n += (double)x[c].r * y[c].r + (double)x[c].i * y[c].i;
    }
    block_sum_store(n, v.partials, blockIdx.x);
}

// One block per system: out[sys * out_stride] = sum of the system's partials
// (fixed order).
__global__ __launch_bounds__(1024) void reduce_batch(const VecSys *sys, const int32_t *active,
                                                     int64_t count_override, double *out,
                                                     int64_t out_stride)
{
    const VecSys v = sys[blockIdx.x];
    if (sys_inactive(v, active)) return;
    __shared__ double sm[1024];
    const int64_t n = count_override > 0 ? count_override : v.nparts;
    double t = 0;
    for (int64_t k = threadIdx.x; k < n; k += 1024) t += v.partials[k];
    sm[threadIdx.x] = t;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x * out_stride] = sm[0];
}

// Per-system CG scalars.  op 0: alpha = gamma / qq;  op 1: beta = gamma_new /
// gamma (0 when the system restarts), gamma = gamma_new.  Inactive systems get
// alpha = beta = 0.
__global__ void cg_scalar_batch(CgScalars *sc, int nsys, int op, const int32_t *active,
                                int32_t *restart, int slot)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsys) return;
    CgScalars &s = sc[j];
    const bool on = !active || active[j];
    const bool rec = on && s.hist && s.nhist < s.hmax;
    if (op == 2) {
        if (on) s.alpha = 0.0;
    } else if (op == 0) {
        s.alpha = (on && s.qq > 0) ? s.gamma / s.qq : 0.0;
        if (rec) s.hist[2 * s.nhist++ + 1] = s.alpha;
        if (slot >= 0) s.aring[slot] = s.alpha;
    } else {
        const bool rs = restart && restart[j];
        s.beta = (on && !rs && s.gamma > 0) ? s.gamma_new / s.gamma : 0.0;
        s.gamma = s.gamma_new;
        if (restart) restart[j] = 0;
        if (rec) s.hist[2 * s.nhist] = s.beta;
    }
}

int sites_per_wave(int Ls) { return 64 / Ls; }

}  // namespace

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point (mobius_dslash_noalloc): one
// statically sized array per GPU, held until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: only the address
// that hipGetSymbolAddress returns for the current device is ever passed to a
// kernel or a copy.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

HopTuning &hop_tuning()
{
    static HopTuning t = [] {
        HopTuning d;
        if (const char *e = std::getenv("MOBIUS_XCD_REMAP")) d.xcd_remap = std::atoi(e);
        if (const char *e = std::getenv("MOBIUS_PREFETCH")) d.prefetch = std::atoi(e);
        if (const char *e = std::getenv("MOBIUS_STAGE_LINKS")) d.stage_links = std::atoi(e);
        if (const char *e = std::getenv("MOBIUS_NT_LINKS")) d.nt_links = std::atoi(e);
        return d;
    }();
    return t;
}

// ---------------------------------------------------------------------------
// launchers

int64_t site_kernel_blocks(const Geometry &g)
{
    const int spw = sites_per_wave(g.Ls);
    const int64_t per_block = (int64_t)spw * WAVES;
    return (g.Vh + per_block - 1) / per_block;
}

int64_t blas_blocks(const Geometry &g) { return (g.N5 + BLAS_BLOCK - 1) / BLAS_BLOCK; }

hipError_t launch_build_geometry(const Geometry &g, const int32_t *packed_of, int32_t *nbr,
                                 hipStream_t st)
{
    Dims D{{g.L[0], g.L[1], g.L[2], g.L[3]}};
    const int64_t n = 2 * g.Vh;
    hipLaunchKernelGGL(build_nbr_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D,
                       g.Vh, g.canon_of, packed_of, nbr);
    return hipGetLastError();
}

hipError_t launch_pack_links(const Geometry &g, int prec, const void *canon, void *packed,
                             hipStream_t st, double sf, double sb)
{
    Dims D{{g.L[0], g.L[1], g.L[2], g.L[3]}};
    const int64_t n = 2 * g.Vh * 8;
    dim3 grid((unsigned)((n + 255) / 256));
    const double2 *c = static_cast<const double2 *>(canon);
    char *o = static_cast<char *>(packed);
    switch (prec) {
    case MOBIUS_F64: hipLaunchKernelGGL(pack_links_kernel<MOBIUS_F64>, grid, dim3(256), 0, st, D, g.V, g.Vh, g.canon_of, c, o, sf, sb); break;
    case MOBIUS_F32: hipLaunchKernelGGL(pack_links_kernel<MOBIUS_F32>, grid, dim3(256), 0, st, D, g.V, g.Vh, g.canon_of, c, o, sf, sb); break;
    case MOBIUS_F16: hipLaunchKernelGGL(pack_links_kernel<MOBIUS_F16>, grid, dim3(256), 0, st, D, g.V, g.Vh, g.canon_of, c, o, sf, sb); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wall_place(const Geometry &g, const void *b4, void *eta5, int nrhs, hipStream_t st)
{
    const int64_t n = (int64_t)nrhs * g.Ls * g.V;
    hipLaunchKernelGGL(wall_place_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.V, g.Ls, n,
                       static_cast<const double2 *>(b4), static_cast<double2 *>(eta5));
    return hipGetLastError();
}

hipError_t launch_wall_read(const Geometry &g, const void *psi5, void *q4, int nrhs, hipStream_t st)
{
    const int64_t n = (int64_t)nrhs * g.V;
    hipLaunchKernelGGL(wall_read_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.V, g.Ls, n,
                       static_cast<const double2 *>(psi5), static_cast<double2 *>(q4));
    return hipGetLastError();
}

hipError_t launch_bulk_assemble(const Geometry &g, const void *psi4, const void *y5, void *Psi5,
                                int nrhs, hipStream_t st)
{
    const int64_t n = (int64_t)nrhs * g.Ls * g.V;
    hipLaunchKernelGGL(bulk_assemble_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.V,
                       g.Ls, n, static_cast<const double2 *>(psi4), static_cast<const double2 *>(y5),
                       static_cast<double2 *>(Psi5));
    return hipGetLastError();
}

hipError_t launch_pack_spinor(const Geometry &g, int prec, const void *canon, void *even, void *odd,
                              int nrhs, hipStream_t st)
{
    const int64_t n = 2 * g.N5;
    dim3 grid((unsigned)((n + 255) / 256));
    const int64_t fb = field_bytes(g, prec);
    for (int r = 0; r < nrhs; ++r) {
        const double2 *c = static_cast<const double2 *>(canon) + (int64_t)r * 2 * g.N5 * 12;
        char *e = static_cast<char *>(even) + r * fb;
        char *o = static_cast<char *>(odd) + r * fb;
        switch (prec) {
        case MOBIUS_F64: hipLaunchKernelGGL(pack_spinor_kernel<MOBIUS_F64>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, c, e, o); break;
        case MOBIUS_F32: hipLaunchKernelGGL(pack_spinor_kernel<MOBIUS_F32>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, c, e, o); break;
        case MOBIUS_F16: hipLaunchKernelGGL(pack_spinor_kernel<MOBIUS_F16>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, c, e, o); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geometry &g, int prec, const void *even, const void *odd,
                                void *canon, int nrhs, hipStream_t st)
{
    const int64_t n = 2 * g.N5;
    dim3 grid((unsigned)((n + 255) / 256));
    const int64_t fb = field_bytes(g, prec);
    for (int r = 0; r < nrhs; ++r) {
        double2 *c = static_cast<double2 *>(canon) + (int64_t)r * 2 * g.N5 * 12;
        const char *e = static_cast<const char *>(even) + r * fb;
        const char *o = static_cast<const char *>(odd) + r * fb;
        switch (prec) {
        case MOBIUS_F64: hipLaunchKernelGGL(unpack_spinor_kernel<MOBIUS_F64>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, e, o, c); break;
        case MOBIUS_F32: hipLaunchKernelGGL(unpack_spinor_kernel<MOBIUS_F32>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, e, o, c); break;
        case MOBIUS_F16: hipLaunchKernelGGL(unpack_spinor_kernel<MOBIUS_F16>, grid, dim3(256), 0, st, g.Vh, g.Ls, g.canon_of, e, o, c); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

namespace {

// dynamic LDS of one block for the staged links: [8][sites per block][record]
template <int P>
size_t link_lds_bytes(int spw, bool rows)
{
    // FP16: the dot2 operand form, or the matrix-core rows (pf 3)
    return (size_t)8 * WAVES * spw * (P == MOBIUS_F16 ? (rows ? LINKROW_REC : LINKH2_REC) : Link<P>::REC);
}

template <int P, bool DAG, int EPI>
void hop_launch(const HopParams &hp0, hipStream_t st)
{
    HopParams hp = hp0;
    const size_t links = hp.stage_links ? link_lds_bytes<P>(hp.spw, hp.pf == 3) : 0;
    size_t dyn = links;
    if constexpr ((EPI & EPI_M5INV) != 0) {
        hp.m5_off = hp.nrhs > 1 ? (int)links : 0;
        dyn = std::max(links, (size_t)hp.m5_off + sizeof(M5Lds<typename Spin<P>::T>));
    }
    const dim3 grid((unsigned)hp.nblocks), blk(BLOCK);
    switch (hp.pf) {
    case 0: hipLaunchKernelGGL((hop_kernel<P, DAG, EPI, 0>), grid, blk, dyn, st, hp); break;
    case 1: hipLaunchKernelGGL((hop_kernel<P, DAG, EPI, 1>), grid, blk, dyn, st, hp); break;
    case 3:
        if constexpr (P == MOBIUS_F16) {
            hipLaunchKernelGGL((hop_kernel<P, DAG, EPI, 3>), grid, blk, dyn, st, hp);
            break;
        }
        [[fallthrough]];
    default: hipLaunchKernelGGL((hop_kernel<P, DAG, EPI, 2>), grid, blk, dyn, st, hp); break;
    }
}

template <int P, bool DAG, int EPI>
void hop_batch_launch(const HopParams *groups, int n, const int64_t *prefix, size_t dyn, int grid,
                      int pf, hipStream_t st)
{
    switch (pf) {
    case 0: hipLaunchKernelGGL((hop_batch_kernel<P, DAG, EPI, 0>), dim3(grid), dim3(BLOCK), dyn, st, groups, n, prefix); break;
    case 1: hipLaunchKernelGGL((hop_batch_kernel<P, DAG, EPI, 1>), dim3(grid), dim3(BLOCK), dyn, st, groups, n, prefix); break;
    case 3:
        if constexpr (P == MOBIUS_F16) {
            hipLaunchKernelGGL((hop_batch_kernel<P, DAG, EPI, 3>), dim3(grid), dim3(BLOCK), dyn, st, groups, n, prefix);
            break;
        }
        [[fallthrough]];
    default: hipLaunchKernelGGL((hop_batch_kernel<P, DAG, EPI, 2>), dim3(grid), dim3(BLOCK), dyn, st, groups, n, prefix); break;
    }
}

// Calls F<P, DAG, EPI>() for the runtime (prec, dag, epi); false if unsupported.
template <template <int, bool, int> class F, class... A>
bool dispatch_hop(int prec, int dag, int epi, A &&...args)
{
#define MOBIUS_EPI_CASES(P, D)                                                                     \
    switch (epi) {                                                                                 \
    case 0: F<P, D, 0>::run(args...); return true;                                                 \
    case EPI_M5INV: F<P, D, EPI_M5INV>::run(args...); return true;                                 \
    case EPI_M5INV | EPI_POSTSUB: F<P, D, EPI_M5INV | EPI_POSTSUB>::run(args...); return true;     \
    case EPI_POSTSUB: F<P, D, EPI_POSTSUB>::run(args...); return true;                             \
    case EPI_M5INV | EPI_POSTSUB | EPI_NORM:                                                       \
        F<P, D, EPI_M5INV | EPI_POSTSUB | EPI_NORM>::run(args...);                                 \
        return true;                                                                               \
    case EPI_PRESUB | EPI_M5INV: F<P, D, EPI_PRESUB | EPI_M5INV>::run(args...); return true;       \
    case EPI_POSTSUB | EPI_NORM: F<P, D, EPI_POSTSUB | EPI_NORM>::run(args...); return true;       \
    case EPI_M5ADD: F<P, D, EPI_M5ADD>::run(args...); return true;                                 \
    case EPI_M5ADD | EPI_PRESUB: F<P, D, EPI_M5ADD | EPI_PRESUB>::run(args...); return true;       \
    case EPI_M5ADD | EPI_PRESUB | EPI_NORM:                                                        \
        F<P, D, EPI_M5ADD | EPI_PRESUB | EPI_NORM>::run(args...);                                  \
        return true;                                                                               \
    case EPI_M5INV | EPI_BMIX:                                                                     \
        if constexpr (!D) F<P, D, EPI_M5INV | EPI_BMIX>::run(args...);                             \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB | EPI_NORM:                                        \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB | EPI_NORM>::run(args...); \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB:                                                   \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5INV | EPI_POSTSUB>::run(args...);           \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_POSTSUB | EPI_NORM:                                                    \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_POSTSUB | EPI_NORM>::run(args...);            \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_POSTSUB:                                                               \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_POSTSUB>::run(args...);                       \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_BMIX:                                                                  \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_BMIX>::run(args...);                          \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5INV | EPI_BMIX:                                                      \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5INV | EPI_BMIX>::run(args...);              \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5INV | EPI_BMIX | EPI_POSTSUB:                                        \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5INV | EPI_BMIX | EPI_POSTSUB>::run(args...); \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5INV | EPI_BMIX | EPI_POSTSUB | EPI_NORM:                             \
        if constexpr (!D)                                                                          \
            F<P, D, EPI_PREMIXED | EPI_M5INV | EPI_BMIX | EPI_POSTSUB | EPI_NORM>::run(args...);   \
        return !D;                                                                                 \
    case EPI_NOBOUT:                                                                               \
        if constexpr (D) F<P, D, EPI_NOBOUT>::run(args...);                                        \
        return D;                                                                                  \
    case EPI_PREMIXED | EPI_M5SUB:                                                                 \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5SUB>::run(args...);                         \
        return !D;                                                                                 \
    case EPI_PREMIXED | EPI_M5SUB | EPI_NORM:                                                      \
        if constexpr (!D) F<P, D, EPI_PREMIXED | EPI_M5SUB | EPI_NORM>::run(args...);              \
        return !D;                                                                                 \
    case EPI_M5SUB:                                                                                \
        if constexpr (D) F<P, D, EPI_M5SUB>::run(args...);                                         \
        return D;                                                                                  \
    case EPI_M5SUB | EPI_NORM:                                                                     \
        if constexpr (D) F<P, D, EPI_M5SUB | EPI_NORM>::run(args...);                              \
        return D;                                                                                  \
    case EPI_NOBOUT | EPI_M5INV | EPI_BMIX:                                                        \
        if constexpr (D) F<P, D, EPI_NOBOUT | EPI_M5INV | EPI_BMIX>::run(args...);                 \
        return D;                                                                                  \
    case EPI_NOBOUT | EPI_POSTSUB:                                                                 \
        if constexpr (D) F<P, D, EPI_NOBOUT | EPI_POSTSUB>::run(args...);                          \
        return D;                                                                                  \
    case EPI_NOBOUT | EPI_POSTSUB | EPI_NORM:                                                      \
        if constexpr (D) F<P, D, EPI_NOBOUT | EPI_POSTSUB | EPI_NORM>::run(args...);               \
        return D;                                                                                  \
    }                                                                                              \
    return false;
    if (dag) {
        if (prec == MOBIUS_F64) { MOBIUS_EPI_CASES(MOBIUS_F64, true) }
        if (prec == MOBIUS_F32) { MOBIUS_EPI_CASES(MOBIUS_F32, true) }
        if (prec == MOBIUS_F16) { MOBIUS_EPI_CASES(MOBIUS_F16, true) }
    } else {
        if (prec == MOBIUS_F64) { MOBIUS_EPI_CASES(MOBIUS_F64, false) }
        if (prec == MOBIUS_F32) { MOBIUS_EPI_CASES(MOBIUS_F32, false) }
        if (prec == MOBIUS_F16) { MOBIUS_EPI_CASES(MOBIUS_F16, false) }
    }
#undef MOBIUS_EPI_CASES
    return false;
}

template <int P, bool D, int E>
struct RunHop {
    static void run(const HopParams &hp, hipStream_t st) { hop_launch<P, D, E>(hp, st); }
};
template <int P, bool D, int E>
struct RunHopBatch {
    static void run(const HopParams *g, int n, const int64_t *prefix, size_t dyn, int grid, int pf,
                    hipStream_t st)
    {
        hop_batch_launch<P, D, E>(g, n, prefix, dyn, grid, pf, st);
    }
};

}  // namespace

size_t m5_epilogue_lds_bytes(int prec)
{
    return prec == MOBIUS_F64 ? sizeof(M5Lds<double>) : sizeof(M5Lds<float>);
}

size_t hop_link_lds_bytes(int prec, int Ls, bool rows)
{
    const int spw = sites_per_wave(Ls);
    switch (prec) {
    case MOBIUS_F64: return link_lds_bytes<MOBIUS_F64>(spw, false);
    case MOBIUS_F32: return link_lds_bytes<MOBIUS_F32>(spw, false);
    default: return link_lds_bytes<MOBIUS_F16>(spw, rows);
    }
}

HopParams make_hop_params(const Geometry &g, const OpCoeffs &c, const void *links,
                          const int32_t *nbr, const HopArgs &a)
{
    HopParams hp{};
    const int64_t lb = (int64_t)8 * g.Vh * link_record_bytes(a.prec);
    hp.links = static_cast<const char *>(links) + (int64_t)a.out_parity * lb;
    hp.nbr = nbr + (int64_t)a.out_parity * 8 * g.Vh;
    hp.in = static_cast<const char *>(a.in);
    hp.out = static_cast<char *>(a.out);
    hp.x = static_cast<const char *>(a.x);
    hp.y = static_cast<const char *>(a.y);
    hp.partials = a.partials;
    hp.active = a.active;
    hp.Vh = g.Vh;
    hp.N5 = g.N5;
    hp.fstride = a.fstride > 0 ? a.fstride : field_bytes(g, a.prec);
    hp.nblocks = site_kernel_blocks(g);
    hp.pstride = a.pstride > 0 ? a.pstride : hp.nblocks;
    hp.Ls = g.Ls;
    hp.spw = sites_per_wave(g.Ls);
    hp.nrhs = a.nrhs;
    const HopTuning &t = a.tune ? *a.tune : hop_tuning();
    hp.remap = t.xcd_remap;
    hp.stage_links = t.stage_links && hop_link_lds_bytes(a.prec, g.Ls, false) <= 64 * 1024;
    hp.nt = t.nt_links;
    hp.pf = prefetch_depth(t, a.prec);
    // matrix-core colour multiply: FP16 with staged links and whole 4-lane
    // groups of one site (Ls divisible by 4)
    if (a.prec == MOBIUS_F16 && t.mfma && hp.stage_links && g.Ls % 4 == 0 &&
        hop_link_lds_bytes(a.prec, g.Ls, true) <= 64 * 1024)
        hp.pf = 3;
    hp.c = c;
    return hp;
}

hipError_t launch_hop(const Geometry &g, const OpCoeffs &c, const void *links, const int32_t *nbr,
                      const HopArgs &a, hipStream_t st)
{
    const HopParams hp = make_hop_params(g, c, links, nbr, a);
    if (!dispatch_hop<RunHop>(a.prec, a.dag, a.epi & ~EPI_BDAG, hp, st)) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_hop_batch(int prec, int dag, int epi, const HopParams *groups_dev, int ngroups,
                            const int64_t *prefix_dev, size_t lds_bytes, int grid, int pf,
                            hipStream_t st)
{
    if (!dispatch_hop<RunHopBatch>(prec, dag, epi & ~EPI_BDAG, groups_dev, ngroups, prefix_dev,
                                   lds_bytes, grid, pf, st))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

namespace {
template <int P>
void m5_launch(int kind, int dag, const char *in, char *out, const Geometry &g, const OpCoeffs &c,
               int64_t blocks, hipStream_t st)
{
    const int spw = sites_per_wave(g.Ls);
    dim3 grid((unsigned)blocks), blk(BLOCK);
    if (kind == 0 && !dag) hipLaunchKernelGGL((m5_kernel<P, false, 0>), grid, blk, 0, st, in, out, g.Vh, g.N5, g.Ls, spw, c);
    if (kind == 0 && dag) hipLaunchKernelGGL((m5_kernel<P, true, 0>), grid, blk, 0, st, in, out, g.Vh, g.N5, g.Ls, spw, c);
    if (kind == 1 && !dag) hipLaunchKernelGGL((m5_kernel<P, false, 1>), grid, blk, 0, st, in, out, g.Vh, g.N5, g.Ls, spw, c);
    if (kind == 1 && dag) hipLaunchKernelGGL((m5_kernel<P, true, 1>), grid, blk, 0, st, in, out, g.Vh, g.N5, g.Ls, spw, c);
}
}  // namespace

hipError_t launch_m5(const Geometry &g, const OpCoeffs &c, int prec, int kind, int dag,
                     const void *in, void *out, int nrhs, hipStream_t st)
{
    const int64_t blocks = site_kernel_blocks(g);
    const int64_t fb = field_bytes(g, prec);
    for (int r = 0; r < nrhs; ++r) {
        const char *i = static_cast<const char *>(in) + r * fb;
        char *o = static_cast<char *>(out) + r * fb;
        switch (prec) {
        case MOBIUS_F64: m5_launch<MOBIUS_F64>(kind, dag, i, o, g, c, blocks, st); break;
        case MOBIUS_F32: m5_launch<MOBIUS_F32>(kind, dag, i, o, g, c, blocks, st); break;
        case MOBIUS_F16: m5_launch<MOBIUS_F16>(kind, dag, i, o, g, c, blocks, st); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_fill_random(int prec, void *ptr, int64_t n5, uint32_t seed, hipStream_t st)
{
    const dim3 grid(2048), blk(256);
    char *p = static_cast<char *>(ptr);
    switch (prec) {
    case MOBIUS_F64: hipLaunchKernelGGL(fill_random_kernel<MOBIUS_F64>, grid, blk, 0, st, p, n5, seed); break;
    case MOBIUS_F32: hipLaunchKernelGGL(fill_random_kernel<MOBIUS_F32>, grid, blk, 0, st, p, n5, seed); break;
    case MOBIUS_F16: hipLaunchKernelGGL(fill_random_kernel<MOBIUS_F16>, grid, blk, 0, st, p, n5, seed); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zero(void *ptr, int64_t bytes, hipStream_t st)
{
    const int64_t n16 = bytes / 16;
    const int64_t ntail = bytes - n16 * 16;
    const int64_t n = n16 > ntail ? n16 : ntail;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       static_cast<uint4 *>(ptr), n16,
                       static_cast<unsigned char *>(ptr) + n16 * 16, ntail);
    return hipGetLastError();
}

hipError_t launch_vec_batch(int kind, int prec, int prec2, const VecSys *sys_dev, int nsys,
                            int64_t max_n5, const int32_t *active, hipStream_t st)
{
    const dim3 grid((unsigned)((max_n5 + BLAS_BLOCK - 1) / BLAS_BLOCK), (unsigned)nsys), blk(BLAS_BLOCK);
#define MOBIUS_L(K) hipLaunchKernelGGL(K, grid, blk, 0, st, sys_dev, active)
#define MOBIUS_P3(KT)                                                                   \
    switch (prec) {                                                                     \
    case MOBIUS_F64: MOBIUS_L((KT<MOBIUS_F64>)); break;                                 \
    case MOBIUS_F32: MOBIUS_L((KT<MOBIUS_F32>)); break;                                 \
    case MOBIUS_F16: MOBIUS_L((KT<MOBIUS_F16>)); break;                                 \
    default: return hipErrorInvalidValue;                                               \
    }
    switch (kind) {
    case VEC_CG_XR:
        if (prec == MOBIUS_F64 && prec2 == MOBIUS_F64) MOBIUS_L((cg_xr_batch<MOBIUS_F64, MOBIUS_F64>));
        else if (prec == MOBIUS_F32 && prec2 == MOBIUS_F32) MOBIUS_L((cg_xr_batch<MOBIUS_F32, MOBIUS_F32>));
        else if (prec == MOBIUS_F16 && prec2 == MOBIUS_F32) MOBIUS_L((cg_xr_batch<MOBIUS_F16, MOBIUS_F32>));
        else return hipErrorInvalidValue;
        break;
    case VEC_AXPBY:
        switch (prec) {
        case MOBIUS_F64: MOBIUS_L((axpby_batch<MOBIUS_F64, false>)); break;
        case MOBIUS_F32: MOBIUS_L((axpby_batch<MOBIUS_F32, false>)); break;
        case MOBIUS_F16: MOBIUS_L((axpby_batch<MOBIUS_F16, false>)); break;
        default: return hipErrorInvalidValue;
        }
        break;
    case VEC_AXPBY_NORM:
        switch (prec) {
        case MOBIUS_F64: MOBIUS_L((axpby_batch<MOBIUS_F64, true>)); break;
        case MOBIUS_F32: MOBIUS_L((axpby_batch<MOBIUS_F32, true>)); break;
        case MOBIUS_F16: MOBIUS_L((axpby_batch<MOBIUS_F16, true>)); break;
        default: return hipErrorInvalidValue;
        }
        break;
    case VEC_NORM2: MOBIUS_P3(norm2_batch) break;
    case VEC_DOT: MOBIUS_P3(dot_batch) break;
    case VEC_PUPD_X:
        if (prec == MOBIUS_F64 && prec2 == MOBIUS_F64) MOBIUS_L((pupd_x_batch<MOBIUS_F64, MOBIUS_F64>));
        else if (prec == MOBIUS_F32 && prec2 == MOBIUS_F32) MOBIUS_L((pupd_x_batch<MOBIUS_F32, MOBIUS_F32>));
        else if (prec == MOBIUS_F16 && prec2 == MOBIUS_F32) MOBIUS_L((pupd_x_batch<MOBIUS_F16, MOBIUS_F32>));
        else return hipErrorInvalidValue;
        break;
    case VEC_XFLUSH:
        if (prec == MOBIUS_F64 && prec2 == MOBIUS_F64) MOBIUS_L((xflush_batch<MOBIUS_F64, MOBIUS_F64>));
        else if (prec == MOBIUS_F32 && prec2 == MOBIUS_F32) MOBIUS_L((xflush_batch<MOBIUS_F32, MOBIUS_F32>));
        else if (prec == MOBIUS_F16 && prec2 == MOBIUS_F32) MOBIUS_L((xflush_batch<MOBIUS_F16, MOBIUS_F32>));
        else return hipErrorInvalidValue;
        break;
    case VEC_ACCUMULATE: MOBIUS_P3(accumulate_batch) break;
    case VEC_CONVERT:
#define MOBIUS_CV(PI)                                                                   \
    switch (prec2) {                                                                    \
    case MOBIUS_F64: MOBIUS_L((convert_batch<PI, MOBIUS_F64>)); break;                  \
    case MOBIUS_F32: MOBIUS_L((convert_batch<PI, MOBIUS_F32>)); break;                  \
    case MOBIUS_F16: MOBIUS_L((convert_batch<PI, MOBIUS_F16>)); break;                  \
    default: return hipErrorInvalidValue;                                               \
    }
        switch (prec) {
        case MOBIUS_F64: MOBIUS_CV(MOBIUS_F64) break;
        case MOBIUS_F32: MOBIUS_CV(MOBIUS_F32) break;
        case MOBIUS_F16: MOBIUS_CV(MOBIUS_F16) break;
        default: return hipErrorInvalidValue;
        }
#undef MOBIUS_CV
        break;
    default: return hipErrorInvalidValue;
    }
#undef MOBIUS_P3
#undef MOBIUS_L
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const VecSys *sys_dev, int nsys, const int32_t *active,
                               int64_t count_override, double *out, int64_t out_stride,
                               hipStream_t st)
{
    hipLaunchKernelGGL(reduce_batch, dim3(nsys), dim3(1024), 0, st, sys_dev, active, count_override,
                       out, out_stride);
    return hipGetLastError();
}

hipError_t launch_rupd_m5inv_batch(int prec, const VecSys *sys_dev, int nsys, int64_t max_blocks,
                                   const int32_t *active, int mode, hipStream_t st)
{
    const dim3 grid((unsigned)max_blocks, (unsigned)nsys), blk(BLOCK);
    switch (prec) {
    case MOBIUS_F64: hipLaunchKernelGGL(rupd_m5inv_batch<MOBIUS_F64>, grid, blk, 0, st, sys_dev, active, mode); break;
    case MOBIUS_F32: hipLaunchKernelGGL(rupd_m5inv_batch<MOBIUS_F32>, grid, blk, 0, st, sys_dev, active, mode); break;
    case MOBIUS_F16: hipLaunchKernelGGL(rupd_m5inv_batch<MOBIUS_F16>, grid, blk, 0, st, sys_dev, active, mode); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cg_scalar_batch(CgScalars *sc, int nsys, int op, const int32_t *active,
                                  int32_t *restart, hipStream_t st, int slot)
{
    if (slot >= RING_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cg_scalar_batch, dim3((nsys + 63) / 64), dim3(64), 0, st, sc, nsys, op,
                       active, restart, slot);
    return hipGetLastError();
}

hipError_t launch_ring_batch(int kind, int prec, int prec2, const VecSys *sys_dev, int nsys,
                             int64_t max_n5, const int32_t *active, int a0, int a1, hipStream_t st)
{
    const dim3 grid((unsigned)((max_n5 + BLAS_BLOCK - 1) / BLAS_BLOCK), (unsigned)nsys), blk(BLAS_BLOCK);
    if (kind == VEC_PUPD_RING) {
        if (a0 < 0 || a0 >= RING_MAX || a1 < 0 || a1 >= RING_MAX) return hipErrorInvalidValue;
        switch (prec) {
        case MOBIUS_F32: hipLaunchKernelGGL(pupd_ring_batch<MOBIUS_F32>, grid, blk, 0, st, sys_dev, active, a0, a1); break;
        case MOBIUS_F16: hipLaunchKernelGGL(pupd_ring_batch<MOBIUS_F16>, grid, blk, 0, st, sys_dev, active, a0, a1); break;
        default: return hipErrorInvalidValue;
        }
    } else if (kind == VEC_XRING) {
        if (a0 < 1 || a0 > RING_MAX || prec2 != MOBIUS_F32) return hipErrorInvalidValue;
        switch (prec) {
        case MOBIUS_F32: hipLaunchKernelGGL((xring_batch<MOBIUS_F32, MOBIUS_F32>), grid, blk, 0, st, sys_dev, active, a0); break;
        case MOBIUS_F16: hipLaunchKernelGGL((xring_batch<MOBIUS_F16, MOBIUS_F32>), grid, blk, 0, st, sys_dev, active, a0); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mobius
