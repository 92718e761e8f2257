// mobius_device.h -- device-side building blocks shared by the HIP kernels
// of libmobius.so: complex arithmetic, buffer-resource loads and stores, the
// packed spinor and link formats (see mobius_internal.h), the spin algebra of
// the chiral basis, the lane <-> (4d site, s) map, the s-direction mixing and
// the I^-1 elimination through LDS, and the FP64 block reduction.
#pragma once

#include "mobius_internal.h"

#include <hip/hip_runtime.h>

namespace mobius {
namespace {

constexpr int WAVES = 4;
constexpr int BLOCK = 64 * WAVES;

// ---------------------------------------------------------------------------
// complex helpers

template <typename T>
struct cx {
    T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
// i * a
template <typename T>
__device__ __forceinline__ cx<T> ti(cx<T> a) { return {-a.i, a.r}; }
// a * b
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// acc + a * b
template <typename T>
__device__ __forceinline__ cx<T> cmadd(cx<T> acc, cx<T> a, cx<T> b)
{
    return {acc.r + a.r * b.r - a.i * b.i, acc.i + a.r * b.i + a.i * b.r};
}
// acc + conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cjmadd(cx<T> acc, cx<T> a, cx<T> b)
{
    return {acc.r + a.r * b.r + a.i * b.i, acc.i + a.r * b.i - a.i * b.r};
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int lane)
{
    return __shfl(v, lane, 64);
}
template <typename T>
__device__ __forceinline__ cx<T> shfl(cx<T> v, int lane)
{
    return {__shfl(v.r, lane, 64), __shfl(v.i, lane, 64)};
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// Every packed array is accessed through a buffer resource descriptor (four
// SGPRs: base, size, format) with a 32-bit per-lane byte offset and a
// wavefront-uniform scalar offset (the chunk or link-element stride).  This
// keeps 64-bit address arithmetic out of the vector registers, and the
// hardware range check turns any access past the end of the array into a
// zero load or a dropped store.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer, CDNA
constexpr int CPOL_NT = 2;              // cache policy bit: non-temporal

// Store-data guard.  Without it, gfx950 code in which a VALU instruction
// rewrote the data registers of a buffer store issued just before it (store
// with an SGPR offset) left wrong values in memory: FP16 fields written by the
// fused CG updates diverged at 12^4 x 16 and larger.  The published wait-state
// rule for stores of more than 64 bits of data (the data registers may not be
// rewritten in the next cycle) exempts buffer stores whose offset is an SGPR,
// and code generation follows the exemption: without the guard this file
// compiles to 11 such stores immediately followed by a VALU write of their
// data registers.  On gfx950 the exempt case corrupts; keeping the data live
// across two wait states after each store removes it; a full vmcnt(0) drain
// does too but costs about 3% in the hop.
// Field stores are non-temporal: a field written by one kernel is hundreds of
// MB and is read back by the next kernel, not from L2, and streaming it past
// the L2 leaves more room there for the neighbour spinors a hop re-reads
// (24^3 x 64, Ls = 12: FP32 hop 3 %, FP16 hop and FP16 solve 2 % faster).
#ifndef MOBIUS_ST_CPOL
#define MOBIUS_ST_CPOL CPOL_NT
#endif
#ifndef MOBIUS_STORE_GUARD
#define MOBIUS_STORE_GUARD(v) asm volatile("s_nop 1" ::"v"(v))
#endif
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ Buf(const void *p, int64_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                              (int)(uint32_t)(bytes > 0xffffffffll ? 0xffffffffll : bytes),
                                              RSRC_WORD3))
    {
    }
    __device__ __forceinline__ u32x4 ld16(uint32_t voff, uint32_t soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    }
    __device__ __forceinline__ u32x2 ld8(uint32_t voff, uint32_t soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    }
    __device__ __forceinline__ uint32_t ld4(uint32_t voff, uint32_t soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
    }
    __device__ __forceinline__ void st16(u32x4 v, uint32_t voff, uint32_t soff) const
    {
        __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, MOBIUS_ST_CPOL);
        MOBIUS_STORE_GUARD(v);
    }
    // non-temporal variants (cache policy NT): data that is not re-read soon
    __device__ __forceinline__ u32x4 ld16_nt(uint32_t voff, uint32_t soff) const
    {
        return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, CPOL_NT);
    }
    __device__ __forceinline__ void st4(uint32_t v, uint32_t voff, uint32_t soff) const
    {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, MOBIUS_ST_CPOL);
        MOBIUS_STORE_GUARD(v);
    }
};

// Wait until every memory instruction this wavefront has issued has completed
// (stores included).
__device__ __forceinline__ void vmem_drain()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Materialise a value in VGPRs at this program point (an empty asm with a
// read-write register operand; no instruction is emitted).  Used to stop the
// compiler from sinking the per-direction arithmetic of the hop below the
// last direction, which would keep every loaded operand live.
template <typename T>
__device__ __forceinline__ void pin(cx<T> &v)
{
    asm volatile("" : "+v"(v.r), "+v"(v.i));
}

// ---------------------------------------------------------------------------
// storage policies for packed spinors: 16-byte chunks over site5

template <int P>
struct Spin;

template <>
struct Spin<MOBIUS_F64> {
    using T = double;
    __host__ __device__ static int64_t bytes(int64_t N5) { return N5 * 192; }
    __device__ static void load(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 t = __builtin_bit_cast(double2, b.ld16(k * 16u, (uint32_t)c * N5 * 16u));
            v[c] = {t.x, t.y};
        }
    }
    __device__ static void store(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
#pragma unroll
        for (int c = 0; c < 12; ++c)
            b.st16(__builtin_bit_cast(u32x4, make_double2(v[c].r, v[c].i)), k * 16u,
                   (uint32_t)c * N5 * 16u);
    }
    __device__ static double store_norm2_q(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
        return store_norm2(b, N5, k, v);
    }
    __device__ static double store_norm2(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
        store(b, N5, k, v);
        double n = 0;
#pragma unroll
        for (int c = 0; c < 12; ++c) n += (double)v[c].r * v[c].r + (double)v[c].i * v[c].i;
        return n;
    }
};

template <>
struct Spin<MOBIUS_F32> {
    using T = float;
    __host__ __device__ static int64_t bytes(int64_t N5) { return N5 * 96; }
    __device__ static void load(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float4 t = __builtin_bit_cast(float4, b.ld16(k * 16u, (uint32_t)c * N5 * 16u));
            v[2 * c] = {t.x, t.y};
            v[2 * c + 1] = {t.z, t.w};
        }
    }
    __device__ static void store(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            b.st16(__builtin_bit_cast(u32x4, make_float4(v[2 * c].r, v[2 * c].i, v[2 * c + 1].r,
                                                         v[2 * c + 1].i)),
                   k * 16u, (uint32_t)c * N5 * 16u);
    }
    __device__ static double store_norm2_q(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
        return store_norm2(b, N5, k, v);
    }
    __device__ static double store_norm2(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
        store(b, N5, k, v);
        double n = 0;
#pragma unroll
        for (int c = 0; c < 12; ++c) n += (double)v[c].r * v[c].r + (double)v[c].i * v[c].i;
        return n;
    }
};

template <>
struct Spin<MOBIUS_F16> {
    using T = float;
    __host__ __device__ static int64_t bytes(int64_t N5) { return N5 * 52; }
    __device__ static void load(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
        const float nrm = __builtin_bit_cast(float, b.ld4(k * 4u, 3u * N5 * 16u));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            half8 t = __builtin_bit_cast(half8, b.ld16(k * 16u, (uint32_t)c * N5 * 16u));
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[4 * c + j] = {nrm * (float)t[2 * j], nrm * (float)t[2 * j + 1]};
        }
    }
    // Encode a site: FP32 max-abs norm, binary16 components scaled by 1/norm
    // (round to nearest even).  decode(encode(v)) is what a later load returns.
    // A site whose largest component is below the smallest normal FP32 value
    // is stored as zero: 1/norm would overflow (the front of a Krylov vector
    // grown from a point source reaches such magnitudes).
    __device__ static float encode(const cx<T> v[12], half8 h[3])
    {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].r), fabsf(v[c].i)));
        if (!(m >= __FLT_MIN__)) m = 0.f;
        // hardware reciprocal (within an ulp of 1/m, far below the binary16 step)
        const float inv = m > 0.f ? __builtin_amdgcn_rcpf(m) : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h[c][2 * j] = (_Float16)(v[4 * c + j].r * inv);
                h[c][2 * j + 1] = (_Float16)(v[4 * c + j].i * inv);
            }
        return m;
    }
    __device__ static void store(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
        half8 h[3];
        const float m = encode(v, h);
#pragma unroll
        for (int c = 0; c < 3; ++c) b.st16(__builtin_bit_cast(u32x4, h[c]), k * 16u, (uint32_t)c * N5 * 16u);
        b.st4(__builtin_bit_cast(uint32_t, m), k * 4u, 3u * N5 * 16u);
    }
    // store, return |stored value|^2 and replace v by the stored value (what a
    // later load returns), all from the encoded registers
    __device__ static double store_norm2_q(const Buf &b, uint32_t N5, uint32_t k, cx<T> v[12])
    {
        half8 h[3];
        const float m = encode(v, h);
#pragma unroll
        for (int c = 0; c < 3; ++c) b.st16(__builtin_bit_cast(u32x4, h[c]), k * 16u, (uint32_t)c * N5 * 16u);
        b.st4(__builtin_bit_cast(uint32_t, m), k * 4u, 3u * N5 * 16u);
        double n = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[4 * c + j] = {m * (float)h[c][2 * j], m * (float)h[c][2 * j + 1]};
                n += (double)v[4 * c + j].r * v[4 * c + j].r + (double)v[4 * c + j].i * v[4 * c + j].i;
            }
        return n;
    }
    // store, and return |stored value|^2 computed from the encoded registers
    __device__ static double store_norm2(const Buf &b, uint32_t N5, uint32_t k, const cx<T> v[12])
    {
        half8 h[3];
        const float m = encode(v, h);
#pragma unroll
        for (int c = 0; c < 3; ++c) b.st16(__builtin_bit_cast(u32x4, h[c]), k * 16u, (uint32_t)c * N5 * 16u);
        b.st4(__builtin_bit_cast(uint32_t, m), k * 4u, 3u * N5 * 16u);
        // m^2 sum h^2: the binary16 squares are exact in FP32 and the 24 of
        // them (each <= 1) are summed by packed dot products with an FP32
        // accumulator (relative rounding below 24 ulp of FP32), then scaled
        // by m^2 in FP64
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const half2v p = {h[c][2 * j], h[c][2 * j + 1]};
                s = __builtin_amdgcn_fdot2(p, p, s, false);
            }
        const double md = (double)m;
        return md * md * (double)s;
    }
};

// link records: [8][Vh] of 9 complex<prec> (padded) for one parity
template <int P>
struct Link;

template <>
struct Link<MOBIUS_F64> {
    using T = double;
    static constexpr int REC = 144;
    __device__ static void from_words(const u32x4 *q, cx<T> u[9])
    {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            double2 t = __builtin_bit_cast(double2, q[e]);
            u[e] = {t.x, t.y};
        }
    }
    __device__ static void load(const Buf &b, uint32_t voff, uint32_t soff, cx<T> u[9])
    {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            double2 t = __builtin_bit_cast(double2, b.ld16(voff + 16u * e, soff));
            u[e] = {t.x, t.y};
        }
    }
};
template <>
struct Link<MOBIUS_F32> {
    using T = float;
    static constexpr int REC = 80;
    __device__ static void from_words(const u32x4 *q, cx<T> u[9])
    {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            float4 t = __builtin_bit_cast(float4, q[k]);
            u[2 * k] = {t.x, t.y};
            if (2 * k + 1 < 9) u[2 * k + 1] = {t.z, t.w};
        }
    }
    __device__ static void load(const Buf &b, uint32_t voff, uint32_t soff, cx<T> u[9])
    {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            float4 t = __builtin_bit_cast(float4, b.ld16(voff + 16u * q, soff));
            u[2 * q] = {t.x, t.y};
            if (2 * q + 1 < 9) u[2 * q + 1] = {t.z, t.w};
        }
    }
};
template <>
struct Link<MOBIUS_F16> {
    using T = float;
    static constexpr int REC = 48;
    __device__ static void from_words(const u32x4 *q, cx<T> u[9])
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            half8 t = __builtin_bit_cast(half8, q[k]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * k + j < 9) u[4 * k + j] = {(float)t[2 * j], (float)t[2 * j + 1]};
        }
    }
    __device__ static void load(const Buf &b, uint32_t voff, uint32_t soff, cx<T> u[9])
    {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            half8 t = __builtin_bit_cast(half8, b.ld16(voff + 16u * q, soff));
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * q + j < 9) u[4 * q + j] = {(float)t[2 * j], (float)t[2 * j + 1]};
        }
    }
    // the record's elements as (re, im) binary16 pairs, unconverted.  (Taken
    // apart as eight halves: extracting single 32-bit lanes of the 128-bit
    // buffer load let the compiler shrink the load to its first lane.)
    __device__ static void raw_from_words(const u32x4 *q, half2v u[9])
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const half8 t = __builtin_bit_cast(half8, q[k]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * k + j < 9) u[4 * k + j] = half2v{t[2 * j], t[2 * j + 1]};
        }
    }
    __device__ static void raw_load(const Buf &b, uint32_t voff, uint32_t soff, half2v u[9])
    {
        u32x4 q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = b.ld16(voff + 16u * k, soff);
        raw_from_words(q, u);
    }
};

// ---------------------------------------------------------------------------
// spin algebra in the chiral basis
//
// g_mu = [[0, A_mu], [A_mu^+, 0]] with A_k = -i sigma_k, A_4 = 1, so for
// psi = (u; l) (u = spins 0,1 = P+ part, l = spins 2,3 = P- part) and a sign
// sigma = +-1:
//   (1 + sigma g_mu) psi = (h ; sigma A_mu^+ h),   h = u + sigma A_mu l,
// i.e. the projector keeps two spin components (a half spinor) and the other
// two are reconstructed after the colour multiply.

// (A_mu l) for the two spin rows, one colour
template <typename T, int MU>
__device__ __forceinline__ void A_apply(cx<T> l0, cx<T> l1, cx<T> &o0, cx<T> &o1)
{
    if constexpr (MU == 0) {        // -i sigma_1: (-i l1, -i l0)
        o0 = {l1.i, -l1.r};
        o1 = {l0.i, -l0.r};
    } else if constexpr (MU == 1) { // -i sigma_2 = [[0,-1],[1,0]]: (-l1, l0)
        o0 = {-l1.r, -l1.i};
        o1 = l0;
    } else if constexpr (MU == 2) { // -i sigma_3: (-i l0, i l1)
        o0 = {l0.i, -l0.r};
        o1 = {-l1.i, l1.r};
    } else {                        // 1
        o0 = l0;
        o1 = l1;
    }
}

// (A_mu^+ w) for the two spin rows, one colour
template <typename T, int MU>
__device__ __forceinline__ void Adag_apply(cx<T> w0, cx<T> w1, cx<T> &o0, cx<T> &o1)
{
    if constexpr (MU == 0) {        // i sigma_1: (i w1, i w0)
        o0 = ti(w1);
        o1 = ti(w0);
    } else if constexpr (MU == 1) { // [[0,1],[-1,0]]: (w1, -w0)
        o0 = w1;
        o1 = {-w0.r, -w0.i};
    } else if constexpr (MU == 2) { // i sigma_3: (i w0, -i w1)
        o0 = ti(w0);
        o1 = {w1.i, -w1.r};
    } else {
        o0 = w0;
        o1 = w1;
    }
}

// One direction of the hopping sum at one lane: acc += (1 + sigma g_mu) M chi,
// M = U (forward) or U^+ (backward), chi the (b5/c5-mixed) neighbour spinor.
template <int P>
__device__ __forceinline__ void load_link(const Buf &links, uint32_t Vh, int d, uint32_t i,
                                          cx<typename Spin<P>::T> u[9])
{
    Link<P>::load(links, i * (uint32_t)Link<P>::REC, (uint32_t)d * Vh * (uint32_t)Link<P>::REC, u);
}


// FP16 direction step in packed binary16 arithmetic with FP32 accumulation.
//
// The half spinor h = al u + bu u_{s-1} + sigma A_mu (al l + bl l_{s+1}) is
// formed from the stored binary16 words with packed half multiply-adds; the
// weights al, bu, bl arrive divided by s = max(|al|, |bu|, |bl|) so that every
// term stays O(1).  The colour multiply M h (M = U or U^+) is a chain of
// packed dot products of two binary16 pairs that accumulate in FP32:
//   Re(U h)  = Ur hr - Ui hi,  Im(U h)  = Ur hi + Ui hr,
//   Re(U* h) = Ur hr + Ui hi,  Im(U* h) = Ur hi - Ui hr,
// whose signs and swaps the link carries (LinkH2), so h enters as formed.
// Finally acc += s (1 + sigma g_mu) (M h) in FP32.
__device__ __forceinline__ float dot2(half2v a, half2v b, float c)
{
    return __builtin_amdgcn_fdot2(a, b, c, false);
}
// the pair with its high half negated (sign bit flip)
__device__ __forceinline__ half2v neg_hi_h2(half2v b)
{
    return __builtin_bit_cast(half2v, __builtin_bit_cast(uint32_t, b) ^ 0x80000000u);
}
__device__ __forceinline__ half2v swap_h2(half2v b)
{
    const uint32_t w = __builtin_bit_cast(uint32_t, b);
    return __builtin_bit_cast(half2v, __builtin_amdgcn_alignbit(w, w, 16u));
}
__device__ __forceinline__ half2v splat_h2(float x)
{
    const _Float16 h = (_Float16)x;
    return half2v{h, h};
}
__device__ __forceinline__ half2v neg_lo_h2(half2v b)
{
    return __builtin_bit_cast(half2v, __builtin_bit_cast(uint32_t, b) ^ 0x00008000u);
}
// chain start: a.lo b.lo + a.hi b.hi with a zero accumulator as an inline
// constant (the builtin with a literal zero costs an extra register move)
__device__ __forceinline__ float dot2_0(half2v a, half2v b)
{
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// An FP16 link in the operand form of the dot2 chains.  For M = U (forward
// hop) or M = U^+ (backward hop) and h_b = (re, im) binary16 pairs,
//   Re (M h)_a = sum_b dot2(pr[a*3+b], h_b),  Im (M h)_a = sum_b dot2(pi[a*3+b], h_b)
// with
//   M = U  : pr_ab = (Re U_ab,  -Im U_ab),  pi_ab = (Im U_ab, Re U_ab)
//   M = U^+: pr_ab = (Re U_ba,   Im U_ba),  pi_ab = (-Im U_ba, Re U_ba).
// The block's links are staged in LDS in this form (one expansion per link
// instead of one sign flip and swap of the half spinor per lane).
struct LinkH2 {
    half2v pr[9], pi[9];
};
constexpr int LINKH2_REC = 80;  // 72 bytes of pairs, padded to 16-byte words

template <bool FWD>
__device__ __forceinline__ void expand_link(const half2v u[9], LinkH2 &x)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const half2v e = FWD ? u[a * 3 + b] : u[b * 3 + a];
            if constexpr (FWD) {
                x.pr[a * 3 + b] = neg_hi_h2(e);
                x.pi[a * 3 + b] = swap_h2(e);
            } else {
                x.pr[a * 3 + b] = e;
                x.pi[a * 3 + b] = neg_lo_h2(swap_h2(e));
            }
        }
}

__device__ __forceinline__ void linkh2_from_words(const u32x4 *q, LinkH2 &x)
{
    half2v w[20];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const half8 t = __builtin_bit_cast(half8, q[k]);
#pragma unroll
        for (int j = 0; j < 4; ++j) w[4 * k + j] = half2v{t[2 * j], t[2 * j + 1]};
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        x.pr[e] = w[e];
        x.pi[e] = w[9 + e];
    }
}

__device__ __forceinline__ void linkh2_to_words(const LinkH2 &x, u32x4 *q)
{
    half2v w[20];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        w[e] = x.pr[e];
        w[9 + e] = x.pi[e];
    }
    w[18] = w[19] = half2v{(_Float16)0, (_Float16)0};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        half8 t;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            t[2 * j] = w[4 * k + j].x;
            t[2 * j + 1] = w[4 * k + j].y;
        }
        q[k] = __builtin_bit_cast(u32x4, t);
    }
}

// The same link as the A operand of the 4x4x4 matrix-core product
// (v_mfma_f32_4x4x4_16b_f16: sixteen independent 4x4 blocks per wavefront;
// lane l supplies row l%4 of block l/4's A and column l%4 of its B, and
// receives column l%4 of its D).  For one 4d site, (M h)_a for the 2 x Ls half
// spinors of its s-lanes is the real 8x8 by 8x1 product
//   rows  (Re0, Im0, Re1, Im1 | Re2, Im2, 0, 0)
//   Re_a = (pr[a*3+0], pr[a*3+1], pr[a*3+2], 0),  Im_a = (pi[a*3+0], ...)
//   B    = (h_0, h_1 | h_2, 0)   (binary16 (re, im) pairs)
// in two row halves (m) and two K halves (k): four products per spin row.
// Four consecutive lanes of one site share the A operand, so the path needs
// Ls divisible by 4.  Staged record: the eight rows, 16 bytes each, and 16
// bytes of padding (a 144-byte stride puts the 16 records that one pass of
// 16 lanes writes in distinct LDS banks; at 128 bytes they fall on eight);
// lane l reads rows l%4 and 4 + l%4.
typedef _Float16 half4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
constexpr int LINKROW_REC = 144;

struct LinkRows {
    half4v a[4];  // (m0, k0), (m0, k1), (m1, k0), (m1, k1) of this lane's rows
};

__device__ __forceinline__ void linkrows_to_words(const LinkH2 &x, u32x4 *q)
{
    auto w = [](half2v v) { return __builtin_bit_cast(uint32_t, v); };
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q[2 * a] = u32x4{w(x.pr[a * 3]), w(x.pr[a * 3 + 1]), w(x.pr[a * 3 + 2]), 0u};
        q[2 * a + 1] = u32x4{w(x.pi[a * 3]), w(x.pi[a * 3 + 1]), w(x.pi[a * 3 + 2]), 0u};
    }
    q[6] = q[7] = u32x4{0u, 0u, 0u, 0u};
}

// One staged FP16 link record: the dot2 operand form, or the matrix-core rows
// (each branch of the caller expands and stores on its own, so that the
// expanded link stays in registers)
template <bool FWD, bool ROWS>
__device__ __forceinline__ void stage_link_f16(const half2v u[9], u32x4 *q)
{
    LinkH2 x;
    expand_link<FWD>(u, x);
    if constexpr (ROWS)
        linkrows_to_words(x, q);
    else
        linkh2_to_words(x, q);
}

// The links of a block's sites, staged in LDS by one cooperative copy so
// that each record crosses the vector-memory pipeline once instead of once
// per s-lane.  Layout [d][site in block][record].
template <int P>
struct LinkSource {
    const Buf *glob;
    const char *lds;   // null: read from global memory
    uint32_t Vh, i, sib, sites_blk;
    __device__ __forceinline__ void get(int d, cx<typename Spin<P>::T> u[9]) const
    {
        constexpr int REC = Link<P>::REC;
        if (lds) {
            const u32x4 *q = reinterpret_cast<const u32x4 *>(lds + ((size_t)d * sites_blk + sib) * REC);
            Link<P>::from_words(q, u);
        } else {
            load_link<P>(*glob, Vh, d, i, u);
        }
    }
    // FP16 links in the dot2 operand form (staged in that form in LDS)
    template <bool FWD>
    __device__ __forceinline__ void get_h2(int d, LinkH2 &x) const
    {
        if (lds) {
            const u32x4 *q = reinterpret_cast<const u32x4 *>(lds + ((size_t)d * sites_blk + sib) * LINKH2_REC);
            linkh2_from_words(q, x);
        } else {
            constexpr int REC = Link<P>::REC;
            half2v u[9];
            Link<P>::raw_load(*glob, i * (uint32_t)REC, (uint32_t)d * Vh * (uint32_t)REC, u);
            expand_link<FWD>(u, x);
        }
    }
    // FP16 links as matrix-core A rows (staged records of LINKROW_REC bytes
    // only); quad = lane % 4
    __device__ __forceinline__ void get_rows(int d, int quad, LinkRows &x) const
    {
        const u32x4 *q = reinterpret_cast<const u32x4 *>(lds + ((size_t)d * sites_blk + sib) * LINKROW_REC);
        const u32x4 r0 = q[quad], r1 = q[4 + quad];
        x.a[0] = __builtin_bit_cast(half4v, u32x2{r0[0], r0[1]});
        x.a[1] = __builtin_bit_cast(half4v, u32x2{r0[2], r0[3]});
        x.a[2] = __builtin_bit_cast(half4v, u32x2{r1[0], r1[1]});
        x.a[3] = __builtin_bit_cast(half4v, u32x2{r1[2], r1[3]});
    }
};

// multiplication of a binary16 pair (re, im) by -i and by +i
__device__ __forceinline__ half2v mul_mi(half2v z) { return half2v{z.y, -z.x}; }
__device__ __forceinline__ half2v mul_pi(half2v z) { return half2v{-z.y, z.x}; }

// h[0..2] = spin row 0, h[3..5] = spin row 1 (colour inner); o holds the 12
// components (spin * 3 + colour) of the site, um the P+ half of slice s-1 and
// lp the P- half of slice s+1.
template <int MU, int SIGMA, bool MIX>
__device__ __forceinline__ void half_spinor_h2(const half2v o[12], const half2v um[6],
                                               const half2v lp[6], half2v al, half2v bu,
                                               half2v bl, half2v h[6])
{
    const half2v sg = splat_h2((float)SIGMA);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // without mixing the only weight is the site norm, restored in FP32
        // by the caller: h is formed from the stored words as they are
        half2v t0 = o[6 + a], t1 = o[9 + a];
        if constexpr (MIX) {
            t0 = al * t0 + bl * lp[a];
            t1 = al * t1 + bl * lp[3 + a];
        }
        half2v A0, A1;  // A_mu (t0; t1)
        if constexpr (MU == 0) {        // -i sigma_1
            A0 = mul_mi(t1);
            A1 = mul_mi(t0);
        } else if constexpr (MU == 1) { // [[0,-1],[1,0]]
            A0 = -t1;
            A1 = t0;
        } else if constexpr (MU == 2) { // -i sigma_3
            A0 = mul_mi(t0);
            A1 = mul_pi(t1);
        } else {
            A0 = t0;
            A1 = t1;
        }
        half2v u0 = o[a], u1 = o[3 + a];
        if constexpr (MIX) {
            u0 = al * u0 + bu * um[a];
            u1 = al * u1 + bu * um[3 + a];
        }
        h[a] = u0 + sg * A0;
        h[3 + a] = u1 + sg * A1;
    }
}

// The colour multiply on the matrix cores (operand layout at LinkRows),
// then the same FP32 reconstruction as link_accumulate_h2.
template <int MU, int SIGMA>
__device__ __forceinline__ void link_accumulate_mfma(const half2v h[6], float s, const LinkRows &x,
                                                     cx<float> acc[12])
{
    const float4v z = {0.f, 0.f, 0.f, 0.f};
    const _Float16 h0 = (_Float16)0;
    cx<float> w[2][3];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
        const half2v *hs = h + 3 * sp;
        const half4v k0 = {hs[0].x, hs[0].y, hs[1].x, hs[1].y};
        const half4v k1 = {hs[2].x, hs[2].y, h0, h0};
        float4v lo = __builtin_amdgcn_mfma_f32_4x4x4f16(x.a[0], k0, z, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_4x4x4f16(x.a[1], k1, lo, 0, 0, 0);
        float4v hi = __builtin_amdgcn_mfma_f32_4x4x4f16(x.a[2], k0, z, 0, 0, 0);
        hi = __builtin_amdgcn_mfma_f32_4x4x4f16(x.a[3], k1, hi, 0, 0, 0);
        w[sp][0] = {lo[0], lo[1]};
        w[sp][1] = {lo[2], lo[3]};
        w[sp][2] = {hi[0], hi[1]};
    }
    const float sg = (float)SIGMA * s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + s * w[0][a];
        acc[3 + a] = acc[3 + a] + s * w[1][a];
        cx<float> o0, o1;
        Adag_apply<float, MU>(w[0][a], w[1][a], o0, o1);
        acc[6 + a] = acc[6 + a] + sg * o0;
        acc[9 + a] = acc[9 + a] + sg * o1;
    }
}

template <int MU, int SIGMA>
__device__ __forceinline__ void link_accumulate_h2(const half2v h[6], float s, const LinkH2 &x,
                                                   cx<float> acc[12])
{
    const float sg = (float)SIGMA * s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float w0r = dot2_0(x.pr[a * 3], h[0]), w0i = dot2_0(x.pi[a * 3], h[0]);
        float w1r = dot2_0(x.pr[a * 3], h[3]), w1i = dot2_0(x.pi[a * 3], h[3]);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            w0r = dot2(x.pr[a * 3 + b], h[b], w0r);
            w0i = dot2(x.pi[a * 3 + b], h[b], w0i);
            w1r = dot2(x.pr[a * 3 + b], h[3 + b], w1r);
            w1i = dot2(x.pi[a * 3 + b], h[3 + b], w1i);
        }
        const cx<float> w0 = {w0r, w0i}, w1 = {w1r, w1i};
        acc[a] = acc[a] + s * w0;
        acc[3 + a] = acc[3 + a] + s * w1;
        cx<float> o0, o1;
        Adag_apply<float, MU>(w0, w1, o0, o1);
        acc[6 + a] = acc[6 + a] + sg * o0;
        acc[9 + a] = acc[9 + a] + sg * o1;
    }
}

// Colour multiply and reconstruction of one direction: acc += (1 + sigma g_mu) M h
// given the half spinor h = (h0; h1) = u + sigma A_mu l, with M = U (forward)
// or U^+ (backward).  u: the link as stored (element a*3+b of U_mu(x) or of
// U_mu(x-mu), whose adjoint the backward term applies).
template <typename T, int MU, bool FWD, int SIGMA>
__device__ __forceinline__ void link_accumulate(const cx<T> h0[3], const cx<T> h1[3],
                                                const cx<T> u[9], cx<T> acc[12])
{
    const T sg = (T)SIGMA;
    cx<T> w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w0[a] = {0, 0};
        w1[a] = {0, 0};
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if constexpr (FWD) {
                w0[a] = cmadd(w0[a], u[a * 3 + b], h0[b]);
                w1[a] = cmadd(w1[a], u[a * 3 + b], h1[b]);
            } else {  // (U^+)_{ab} = conj(U_ba)
                w0[a] = cjmadd(w0[a], u[b * 3 + a], h0[b]);
                w1[a] = cjmadd(w1[a], u[b * 3 + a], h1[b]);
            }
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + w0[a];
        acc[3 + a] = acc[3 + a] + w1[a];
        cx<T> o0, o1;
        Adag_apply<T, MU>(w0[a], w1[a], o0, o1);
        acc[6 + a] = acc[6 + a] + sg * o0;
        acc[9 + a] = acc[9 + a] + sg * o1;
    }
}

// One direction from a full (already b5/c5-mixed) spinor chi.
template <int P, int MU, bool FWD, int SIGMA>
__device__ __forceinline__ void hop_dir(const cx<typename Spin<P>::T> chi[12],
                                        const cx<typename Spin<P>::T> u[9],
                                        cx<typename Spin<P>::T> acc[12])
{
    using T = typename Spin<P>::T;
    const T sg = (T)SIGMA;
    cx<T> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<T> o0, o1;
        A_apply<T, MU>(chi[6 + a], chi[9 + a], o0, o1);
        h0[a] = chi[a] + sg * o0;
        h1[a] = chi[3 + a] + sg * o1;
    }
    link_accumulate<T, MU, FWD, SIGMA>(h0, h1, u, acc);
}

// ---------------------------------------------------------------------------
// FP16 direction step without dequantising the spinor: the raw binary16
// words of the neighbour (and, for the b5/c5 mixing, of its s-1 and s+1
// slices, fetched from the neighbouring lanes) enter the half spinor through
// packed binary16 multiply-adds whose scalar factors fold the per-site norms
// and the mixing weights (see half_spinor_h2):
//   h = al u_s + bu u_{s-1} + sigma A (al l_s + bl l_{s+1}),
//   al = b5 n_s, bu = c5 f n_{s-1}, bl = c5 f' n_{s+1}  (f, f' = -mf on the wrap).

struct RawH {
    half2v c[12];  // complex components as (re, im) binary16 pairs
    float n;       // per-site norm
};

__device__ __forceinline__ void load_raw_f16(const Buf &b, uint32_t N5, uint32_t k, RawH &r)
{
    r.n = __builtin_bit_cast(float, b.ld4(k * 4u, 3u * N5 * 16u));
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const half8 t = __builtin_bit_cast(half8, b.ld16(k * 16u, (uint32_t)q * N5 * 16u));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            half2v h;
            h.x = t[2 * j];
            h.y = t[2 * j + 1];
            r.c[4 * q + j] = h;
        }
    }
}

__device__ __forceinline__ half2v shfl_h2(half2v v, int lane)
{
    return __builtin_bit_cast(half2v, __shfl((int)__builtin_bit_cast(uint32_t, v), lane, 64));
}

struct SiteMap {
    int lane, wave, g, s;
    bool site_ok;
    int64_t i;   // packed 4d site (clamped to a valid index)
    int lm, lp;  // lanes holding s-1 and s+1 of the same site (cyclic)
};

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8), each with its own L2.  With remap on, the blocks an XCD receives
// cover one contiguous range of sites, so the neighbours a block reads were
// mostly fetched into the same L2 by the blocks just before it.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ int64_t logical_block(int remap)
{
    const int64_t b = blockIdx.x;
    if (!remap) return b;
    const int64_t nb = gridDim.x;
    const int64_t q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int64_t x = b % NUM_XCD, c = b / NUM_XCD;
    return x * q + (x < r ? x : r) + c;
}

__device__ __forceinline__ SiteMap site_map_lb(int Ls, int spw, int64_t Vh, int64_t lb)
{
    SiteMap m;
    m.lane = threadIdx.x & 63;
    m.wave = threadIdx.x >> 6;
    m.g = m.lane / Ls;
    m.s = m.lane - m.g * Ls;
    int64_t i = (lb * WAVES + m.wave) * spw + m.g;
    m.site_ok = (m.g < spw) && (i < Vh);
    m.i = m.site_ok ? i : 0;
    const int base = m.g * Ls;
    m.lm = base + (m.s == 0 ? Ls - 1 : m.s - 1);
    m.lp = base + (m.s == Ls - 1 ? 0 : m.s + 1);
    return m;
}

__device__ __forceinline__ SiteMap site_map(int Ls, int spw, int64_t Vh, int remap = 0)
{
    return site_map_lb(Ls, spw, Vh, logical_block(remap));
}

template <typename T>
struct Coef {
    T b5, c5, mf, Mp, Mm, a, mu, inv_Mp, inv_den;
    const double *ls;  // per-slice table (null: constant coefficients)
};

template <typename T>
__device__ __forceinline__ Coef<T> make_coef(const OpCoeffs &c)
{
    return {(T)c.b5, (T)c.c5, (T)c.mf, (T)c.Mp, (T)c.Mm, (T)c.a, (T)c.mu, (T)c.inv_Mp,
            (T)c.inv_den, c.ls};
}

// Weights of one lane of X + Y C5 (forward) or X + C5^+ Y (adjoint), with
// (X, Y) = (b5, c5) for B or (M+, M-) for I: a is the lane's own X, bu and bl
// the Y of the rows the P+ and P- parts belong to -- the lane's own row in
// the forward form, the source rows s+1 and s-1 in the adjoint (Y is a
// coefficient of the row of D_DW, so the adjoint carries it to the column).
template <typename T>
struct MixW {
    T a, bu, bl;
};

template <typename T>
__device__ __forceinline__ MixW<T> mix_w(const Coef<T> &k, bool minv, const SiteMap &m, int Ls,
                                         bool adjoint)
{
    const T X = minv ? k.Mp : k.b5, Y = minv ? k.Mm : k.c5;
    if (!k.ls) return {X, Y, Y};
    const int ox = minv ? LS_MP : LS_B5;
    const double *t = k.ls;
    const T a = (T)t[m.s * LSC + ox];
    if (!adjoint) {
        const T y = (T)t[m.s * LSC + ox + 1];
        return {a, y, y};
    }
    const int su = m.s == Ls - 1 ? 0 : m.s + 1, sl = m.s == 0 ? Ls - 1 : m.s - 1;
    return {a, (T)t[su * LSC + ox + 1], (T)t[sl * LSC + ox + 1]};
}

// C5 mixing in s from the lanes of the same 4d site, constant coefficients.
//   forward  (C5 v)_s  = P+ v_{s-1} + P- v_{s+1}
//   adjoint  (C5^+ v)_s = P+ v_{s+1} + P- v_{s-1}
// wrapped neighbours carry -mf.  Returns alpha * v + beta * C5(^+) v.
template <typename T>
__device__ __forceinline__ void mix_s(cx<T> v[12], T alpha, T beta, T mf, const SiteMap &m, int Ls,
                                      bool adjoint)
{
    const int src_up = adjoint ? m.lp : m.lm;  // lane whose P+ part we take
    const int src_lo = adjoint ? m.lm : m.lp;  // lane whose P- part we take
    const bool wrap_up = adjoint ? (m.s == Ls - 1) : (m.s == 0);
    const bool wrap_lo = adjoint ? (m.s == 0) : (m.s == Ls - 1);
    const T fu = beta * (wrap_up ? -mf : (T)1);
    const T fl = beta * (wrap_lo ? -mf : (T)1);
    cx<T> up[6], lo[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        up[c] = shfl(v[c], src_up);
        lo[c] = shfl(v[6 + c], src_lo);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        v[c] = alpha * v[c] + fu * up[c];
        v[6 + c] = alpha * v[6 + c] + fl * lo[c];
    }
}

// The same with per-lane weights: w.a v + (w.bu P+ + w.bl P-) C5(^+) v.
template <typename T>
__device__ __forceinline__ void mix_s(cx<T> v[12], MixW<T> w, T mf, const SiteMap &m, int Ls,
                                      bool adjoint)
{
    const int src_up = adjoint ? m.lp : m.lm;  // lane whose P+ part we take
    const int src_lo = adjoint ? m.lm : m.lp;  // lane whose P- part we take
    const bool wrap_up = adjoint ? (m.s == Ls - 1) : (m.s == 0);
    const bool wrap_lo = adjoint ? (m.s == 0) : (m.s == Ls - 1);
    const T alpha = w.a;
    const T fu = w.bu * (wrap_up ? -mf : (T)1);
    const T fl = w.bl * (wrap_lo ? -mf : (T)1);
    cx<T> up[6], lo[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        up[c] = shfl(v[c], src_up);
        lo[c] = shfl(v[6 + c], src_lo);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        v[c] = alpha * v[c] + fu * up[c];
        v[6 + c] = alpha * v[6 + c] + fl * lo[c];
    }
}

// I^-1 (or I^-+) of Sec. 3 on the Ls lanes of each 4d site, through LDS.
// I^-1 = A^-1 P- + A^-T P+;  I^-+ = A^-T P- + A^-1 P+  (A real).
// Lane (g, s) of a site solves component c = s, s + Ls, ... by the paper's
// elimination on the fly:
//   A^-1 b:  psi_Ls = (b_Ls + mu sum_{s<Ls} (-a)^(s-1) b_s) / (M+ (1 - mu (-a)^(Ls-1)))
//            psi_s  = b_s / M+ - a psi_{s+1}
//   A^-T b:  psi_1  = (b_1 + mu sum_{s>1} (-a)^(Ls-s) b_s) / (same)
//            psi_s  = b_s / M+ - a psi_{s-1}
template <typename T>
struct M5Lds {
    static constexpr int STRIDE = 13;  // complex per lane (12 + 1 pad)
    cx<T> buf[WAVES][64 * STRIDE];
};

template <typename T>
__device__ __forceinline__ void m5inv_lanes(cx<T> r[12], const Coef<T> &k, const SiteMap &m, int Ls,
                                            bool dag, M5Lds<T> &lds)
{
    // lane coordinates recomputed here (opaque to common-subexpression
    // elimination, same mapping as m) so that no address of this step is held
    // in a register across the caller's main loop
    (void)m;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = (int)(tid & 63u), wave = (int)(tid >> 6), g = lane / Ls, s0 = lane - g * Ls;
    cx<T> *w = lds.buf[wave];
    constexpr int ST = M5Lds<T>::STRIDE;
#pragma unroll
    for (int c = 0; c < 12; ++c) w[lane * ST + c] = r[c];
    __syncthreads();
    if (k.ls && g * Ls + Ls <= 64) {
        // s-dependent coefficients: the cyclic bidiagonal form of each
        // chirality (P-: M-(t) at (t, t+1) and -m M-(Ls) at (Ls, 1); P+: M-(t)
        // at (t, t-1) and -m M-(1) at (1, Ls); transposed for I^+), solved by
        // the same elimination with per-row ratios: the unknown at the far end
        // from the running sum S and product g, then back-substitution.
        const int base = g * Ls;
        const double *tb = k.ls;
        const T corner_m = -k.mf * (T)tb[(Ls - 1) * LSC + LS_MM];
        const T corner_p = -k.mf * (T)tb[LS_MM];
        for (int c = s0; c < 12; c += Ls) {
            const bool minus = c >= 6;
            const bool upper = minus != dag;
            const T kc = minus ? corner_m : corner_p;
            // off-diagonal element of row t: forward M-(t); adjoint M-(t-1)
            // (P-) or M-(t+1) (P+)
            const int sh = !dag ? 0 : (minus ? -1 : 1);
            cx<T> S = {0, 0};
            T gg = (T)1;
            if (upper) {
                for (int t = 0; t < Ls - 1; ++t) {
                    const T id = (T)tb[t * LSC + LS_INV_MP], e = (T)tb[(t + sh) * LSC + LS_MM];
                    S = S + (gg * id) * w[(base + t) * ST + c];
                    gg = -gg * e * id;
                }
                const T dl = (T)tb[(Ls - 1) * LSC + LS_MP];
                cx<T> psi = ((T)1 / (dl + kc * gg)) * (w[(base + Ls - 1) * ST + c] - kc * S);
                w[(base + Ls - 1) * ST + c] = psi;
                for (int t = Ls - 2; t >= 0; --t) {
                    const T id = (T)tb[t * LSC + LS_INV_MP], e = (T)tb[(t + sh) * LSC + LS_MM];
                    psi = id * (w[(base + t) * ST + c] - e * psi);
                    w[(base + t) * ST + c] = psi;
                }
            } else {
                for (int t = Ls - 1; t > 0; --t) {
                    const T id = (T)tb[t * LSC + LS_INV_MP], e = (T)tb[(t + sh) * LSC + LS_MM];
                    S = S + (gg * id) * w[(base + t) * ST + c];
                    gg = -gg * e * id;
                }
                const T d0 = (T)tb[LS_MP];
                cx<T> psi = ((T)1 / (d0 + kc * gg)) * (w[base * ST + c] - kc * S);
                w[base * ST + c] = psi;
                for (int t = 1; t < Ls; ++t) {
                    const T id = (T)tb[t * LSC + LS_INV_MP], e = (T)tb[(t + sh) * LSC + LS_MM];
                    psi = id * (w[(base + t) * ST + c] - e * psi);
                    w[(base + t) * ST + c] = psi;
                }
            }
        }
    } else if (g * Ls + Ls <= 64) {
        // Both recurrences walk the slices in order; the loads of four slices
        // are issued together (a load never depends on the recurrence), so a
        // wave waits for LDS once per four steps instead of once per step.
        // The arithmetic and its order are those of the plain loop.
        const int base = g * Ls;
        for (int c = s0; c < 12; c += Ls) {
            const bool plus = c < 6;
            const bool transpose = plus != dag;
            const T na = -k.a;
            // slice t of this component; dt = -1 walks down from Ls - 2, +1 up from 1
            const int dt = transpose ? 1 : -1;
            const int t0 = transpose ? 1 : Ls - 2;   // first slice of both loops
            const int tl = transpose ? 0 : Ls - 1;   // the slice solved first
            cx<T> *col = w + base * ST + c;
            cx<T> sum = {0, 0};
            int n = Ls - 1, t = t0;
            for (; n >= 4; n -= 4, t += 4 * dt) {
                const cx<T> w0 = col[t * ST], w1 = col[(t + dt) * ST], w2 = col[(t + 2 * dt) * ST],
                            w3 = col[(t + 3 * dt) * ST];
                sum = w0 + na * sum;
                sum = w1 + na * sum;
                sum = w2 + na * sum;
                sum = w3 + na * sum;
            }
            for (; n > 0; --n, t += dt) sum = col[t * ST] + na * sum;
            cx<T> psi = k.inv_den * (col[tl * ST] + k.mu * sum);
            col[tl * ST] = psi;
            n = Ls - 1;
            t = t0;
            for (; n >= 4; n -= 4, t += 4 * dt) {
                const cx<T> w0 = col[t * ST], w1 = col[(t + dt) * ST], w2 = col[(t + 2 * dt) * ST],
                            w3 = col[(t + 3 * dt) * ST];
                psi = k.inv_Mp * w0 - k.a * psi;
                col[t * ST] = psi;
                psi = k.inv_Mp * w1 - k.a * psi;
                col[(t + dt) * ST] = psi;
                psi = k.inv_Mp * w2 - k.a * psi;
                col[(t + 2 * dt) * ST] = psi;
                psi = k.inv_Mp * w3 - k.a * psi;
                col[(t + 3 * dt) * ST] = psi;
            }
            for (; n > 0; --n, t += dt) {
                psi = k.inv_Mp * col[t * ST] - k.a * psi;
                col[t * ST] = psi;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 12; ++c) r[c] = w[lane * ST + c];
}

// FP64 block reduction of one value per thread -> partials[slot]
__device__ __forceinline__ void block_sum_store(double v, double *partials, int64_t slot)
{
    __shared__ double red[WAVES];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) t += red[w];
        partials[slot] = t;
    }
    __syncthreads();  // red[] may be reused by the next call in this block
}

template <typename T>
__device__ __forceinline__ double site_norm2(const cx<T> r[12])
{
    double n = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) n += (double)r[c].r * r[c].r + (double)r[c].i * r[c].i;
    return n;
}

}  // namespace
}  // namespace mobius
