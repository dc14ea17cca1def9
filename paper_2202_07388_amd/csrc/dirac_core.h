// dirac_core.h -- per-site building blocks of the Wilson-clover stencil: spin
// projection with (1 +- gamma_mu) in the chiral basis, link rebuild and multiply, and the
// 6x6 Hermitian clover blocks. Used by the full-lattice operator and by the SAP block
// solver.
#pragma once

#include "qdw_internal.h"

namespace qdw {

// spin projection h = (1 + SG gamma_MU) psi, upper two spins (chiral basis)
template <typename R, int MU, int SG>
__device__ __forceinline__ void project(const cx<R> s[12], cx<R> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> a0 = s[c], a1 = s[3 + c], a2 = s[6 + c], a3 = s[9 + c];
        if (MU == 0) {
            h[c] = SG > 0 ? a0 - a2 : a0 + a2;
            h[3 + c] = SG > 0 ? a1 - a3 : a1 + a3;
        } else if (MU == 1) {
            h[c] = SG > 0 ? a0 - times_i(a3) : a0 + times_i(a3);
            h[3 + c] = SG > 0 ? a1 - times_i(a2) : a1 + times_i(a2);
        } else if (MU == 2) {
            h[c] = SG > 0 ? a0 - a3 : a0 + a3;
            h[3 + c] = SG > 0 ? a1 + a2 : a1 - a2;
        } else {
            h[c] = SG > 0 ? a0 - times_i(a2) : a0 + times_i(a2);
            h[3 + c] = SG > 0 ? a1 + times_i(a3) : a1 - times_i(a3);
        }
    }
}

// acc += full spinor rebuilt from the projected, transported half spinor w
template <typename R, int MU, int SG>
__device__ __forceinline__ void expand_add(const cx<R> w[6], cx<R> acc[12])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> w0 = w[c], w1 = w[3 + c];
        acc[c] = acc[c] + w0;
        acc[3 + c] = acc[3 + c] + w1;
        if (MU == 0) {
            acc[6 + c] = SG > 0 ? acc[6 + c] - w0 : acc[6 + c] + w0;
            acc[9 + c] = SG > 0 ? acc[9 + c] - w1 : acc[9 + c] + w1;
        } else if (MU == 1) {
            acc[6 + c] = SG > 0 ? acc[6 + c] + times_i(w1) : acc[6 + c] - times_i(w1);
            acc[9 + c] = SG > 0 ? acc[9 + c] + times_i(w0) : acc[9 + c] - times_i(w0);
        } else if (MU == 2) {
            acc[6 + c] = SG > 0 ? acc[6 + c] + w1 : acc[6 + c] - w1;
            acc[9 + c] = SG > 0 ? acc[9 + c] - w0 : acc[9 + c] + w0;
        } else {
            acc[6 + c] = SG > 0 ? acc[6 + c] + times_i(w0) : acc[6 + c] - times_i(w0);
            acc[9 + c] = SG > 0 ? acc[9 + c] - times_i(w1) : acc[9 + c] + times_i(w1);
        }
    }
}

// FP64 links keep d = det U = exp(3 i theta) (|d| = 1) in one double: the component of
// smaller magnitude, with its two lowest mantissa bits replaced by which component it is
// (bit 0: 1 = imaginary) and the sign of the other one (bit 1: 1 = negative); the other
// component is sqrt(1 - c^2), well conditioned since |c| <= 1/sqrt(2). The two bits cost
// at most 3 ulp of c.
__host__ __device__ __forceinline__ double encode_phase(double re, double im)
{
    const bool use_im = fabs(im) < fabs(re);
    const double c = use_im ? im : re;
    const double other = use_im ? re : im;
    unsigned long long b;
    __builtin_memcpy(&b, &c, 8);
    b = (b & ~3ull) | (use_im ? 1ull : 0ull) | (other < 0.0 ? 2ull : 0ull);
    double out;
    __builtin_memcpy(&out, &b, 8);
    return out;
}

__device__ __forceinline__ cx<double> decode_phase(double e)
{
    unsigned long long b;
    __builtin_memcpy(&b, &e, 8);
    const bool use_im = b & 1ull, neg = b & 2ull;
    b &= ~3ull;
    double c;
    __builtin_memcpy(&c, &b, 8);
    double o = sqrt(fmax(0.0, 1.0 - c * c));
    if (neg) o = -o;
    return use_im ? cx<double>{o, c} : cx<double>{c, o};
}

// link (par, i, mu): rows 0, 1 of the U(3) matrix U (6 complex) and d = det U
template <int P>
__device__ __forceinline__ void load_link(const void* links, const void* dets, int Vh, int par,
                                          int i, int mu, cx<typename Traits<P>::real> u[6],
                                          cx<typename Traits<P>::real>& d)
{
    using T = Traits<P>;
    using R = typename T::real;
    const long row = (long)(par * 4 + mu);
    if constexpr (P == F64 || P == F32) {
#pragma unroll
        for (int k = 0; k < T::LINK_CHUNKS; ++k) {
            Chunk<P> c = load_chunk_cached<P>(links, chunk_at(Vh, T::LINK_CHUNKS, row, k, i));
#pragma unroll
            for (int j = 0; j < T::PER_CHUNK / 2; ++j)
                u[k * (T::PER_CHUNK / 2) + j] = {c.v[2 * j], c.v[2 * j + 1]};
        }
        if constexpr (P == F64) {
            d = decode_phase(((const double*)dets)[row * Vh + i]);
        } else {
            const R* dp = (const R*)dets + 2 * (row * Vh + i);
            d = {dp[0], dp[1]};
        }
    } else {
        Chunk<P> c0 = load_chunk_cached<P>(links, chunk_at(Vh, 2, row, 0, i));
        Chunk<P> c1 = load_chunk_cached<P>(links, chunk_at(Vh, 2, row, 1, i));
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = {to_real<P>(c0.v[2 * j]), to_real<P>(c0.v[2 * j + 1])};
        u[4] = {to_real<P>(c1.v[0]), to_real<P>(c1.v[1])};
        u[5] = {to_real<P>(c1.v[2]), to_real<P>(c1.v[3])};
        d = {to_real<P>(c1.v[4]), to_real<P>(c1.v[5])};
    }
}

// w = U h (DAGGER: U^+ h) for both spin components of the half spinor h; row 2 of U is
// rebuilt as d * conj(row0 x row1)
template <typename R, bool DAGGER>
__device__ __forceinline__ void su3_mul(const cx<R> u[6], cx<R> d, const cx<R> h[6], cx<R> w[6])
{
    const cx<R> r2[3] = {d * conj_(cmadd(u[1] * u[5], -u[2], u[4])),
                         d * conj_(cmadd(u[2] * u[3], -u[0], u[5])),
                         d * conj_(cmadd(u[0] * u[4], -u[1], u[3]))};
    const cx<R> m[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const cx<R> h0 = h[3 * a], h1 = h[3 * a + 1], h2 = h[3 * a + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (!DAGGER)
                w[3 * a + r] = cmadd(cmadd(m[3 * r] * h0, m[3 * r + 1], h1), m[3 * r + 2], h2);
            else
                w[3 * a + r] = cmadd_conj(cmadd_conj(cmul_conj(m[r], h0), m[3 + r], h1), m[6 + r], h2);
        }
    }
}

// o = A v for one 6x6 Hermitian block given as 6 real diagonal entries followed by the
// 15 complex upper-triangle entries (row-major)
template <typename R>
__device__ __forceinline__ void herm6_apply(const R* a, const cx<R>* v, cx<R>* o)
{
#pragma unroll
    for (int r = 0; r < 6; ++r) o[r] = scale(v[r], a[r]);
    int n = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int q = r + 1; q < 6; ++q) {
            const cx<R> e = {a[6 + 2 * n], a[6 + 2 * n + 1]};
            o[r] = cmadd(o[r], e, v[q]);
            o[q] = cmadd_conj(o[q], e, v[r]);
            ++n;
        }
}

// acc = A_+ psi_+ (+) A_- psi_- for the two 6x6 Hermitian chirality blocks of site (par, i)
template <int P>
__device__ __forceinline__ void clover_apply(const void* clover, int Vh, int par, int i,
                                             const cx<typename Traits<P>::real> s[12],
                                             cx<typename Traits<P>::real> acc[12])
{
    using T = Traits<P>;
    using R = typename T::real;
    const long base = chunk_at(Vh, T::CLOVER_CHUNKS, par, 0, i);
    if constexpr (T::PER_CHUNK == 8) {
        // 16-bit storage: the 72 reals are 9 chunks; block 0 ends inside chunk 4
        R a[72];
#pragma unroll
        for (int k = 0; k < T::CLOVER_CHUNKS; ++k) {
            Chunk<P> c = load_chunk<P>(clover, base + (long)k * kSB);
#pragma unroll
            for (int j = 0; j < 8; ++j) a[8 * k + j] = to_real<P>(c.v[j]);
        }
        herm6_apply<R>(a, s, acc);
        herm6_apply<R>(a + 36, s + 6, acc + 6);
    } else {
        constexpr int CPB = T::CLOVER_CHUNKS / 2;  // chunks per block
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            R a[36];
#pragma unroll
            for (int k = 0; k < CPB; ++k) {
                Chunk<P> c = load_chunk<P>(clover, base + (long)(b * CPB + k) * kSB);
#pragma unroll
                for (int j = 0; j < T::PER_CHUNK; ++j) a[k * T::PER_CHUNK + j] = to_real<P>(c.v[j]);
            }
            herm6_apply<R>(a, s + 6 * b, acc + 6 * b);
        }
    }
}

// Compact clover term. In the chiral basis every sigma_{mu nu} acts on the two spins of a
// chirality as a traceless 2x2 matrix, so a chirality block of A is
//     A_+- = c 1 + [[ H, b ], [ b^+, -H ]]      (c = 4 + m0; H Hermitian 3x3, b complex 3x3)
// in its two spins' colour blocks: 27 reals per block instead of the 36 of a general 6x6
// Hermitian block, exactly. Stored reals per site (54; 32- and 16-bit rows padded to 56):
//     0-2 H+ diagonal, 3-5 H- diagonal, 6-11 H+ upper (01, 02, 12), 12-29 b+ (row-major),
//     30-35 H- upper, 36-53 b-.
constexpr int kCl54F64Chunks = 27, kCl54F32Chunks = 14, kCl54F16Chunks = 7;
template <int P> struct Cl54Chunks;
template <> struct Cl54Chunks<F64> { static constexpr int n = kCl54F64Chunks; };
template <> struct Cl54Chunks<F32> { static constexpr int n = kCl54F32Chunks; };
template <> struct Cl54Chunks<F16S> { static constexpr int n = kCl54F16Chunks; };
template <> struct Cl54Chunks<BF16S> { static constexpr int n = kCl54F16Chunks; };

// o = H v for H Hermitian 3x3 from its real diagonal hd[3] and upper entries hu[6]
template <typename R>
__device__ __forceinline__ void herm3_apply(const R* hd, const R* hu, const cx<R>* v, cx<R>* o)
{
    const cx<R> h01 = {hu[0], hu[1]}, h02 = {hu[2], hu[3]}, h12 = {hu[4], hu[5]};
    o[0] = cmadd(cmadd(scale(v[0], hd[0]), h01, v[1]), h02, v[2]);
    o[1] = cmadd(cmadd_conj(scale(v[1], hd[1]), h01, v[0]), h12, v[2]);
    o[2] = cmadd_conj(cmadd_conj(scale(v[2], hd[2]), h02, v[0]), h12, v[1]);
}

// acc (6) = (c + [[H, b], [b^+, -H]]) s (6) for one chirality block
template <typename R>
__device__ __forceinline__ void cl54_block(R c, const R* hd, const R* hu, const R* b,
                                           const cx<R>* s, cx<R>* acc)
{
    cx<R> hu_[3], hl_[3];
    herm3_apply<R>(hd, hu, s, hu_);
    herm3_apply<R>(hd, hu, s + 3, hl_);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        // c s + H s_u + b s_l ; c s + b^+ s_u - H s_l
        cx<R> a0 = hu_[r], a1 = hl_[r];
        a0 = {fmar(c, s[r].re, a0.re), fmar(c, s[r].im, a0.im)};
        a1 = {fmar(c, s[3 + r].re, -a1.re), fmar(c, s[3 + r].im, -a1.im)};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a0 = cmadd(a0, cx<R>{b[2 * (3 * r + q)], b[2 * (3 * r + q) + 1]}, s[3 + q]);
            a1 = cmadd_conj(a1, cx<R>{b[2 * (3 * q + r)], b[2 * (3 * q + r) + 1]}, s[q]);
        }
        acc[r] = a0;
        acc[3 + r] = a1;
    }
}

// acc = A s for site (par, i) from the compact clover array (see above)
template <int P>
__device__ __forceinline__ void clover54_apply(const void* cl, int Vh, int par, int i,
                                               typename Traits<P>::real c,
                                               const cx<typename Traits<P>::real> s[12],
                                               cx<typename Traits<P>::real> acc[12])
{
    using T = Traits<P>;
    using R = typename T::real;
    constexpr int NC = Cl54Chunks<P>::n;
    const long base = chunk_at(Vh, NC, par, 0, i);
    if constexpr (P == F64) {
        // diagonals of both blocks first, then one block at a time (fewer live registers)
        R d[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Chunk<P> ch = load_chunk<P>(cl, base + (long)k * kSB);
            d[2 * k] = ch.v[0];
            d[2 * k + 1] = ch.v[1];
        }
#pragma unroll
        for (int blk = 0; blk < 2; ++blk) {
            R a[24];
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                Chunk<P> ch = load_chunk<P>(cl, base + (long)(3 + 12 * blk + k) * kSB);
                a[2 * k] = ch.v[0];
                a[2 * k + 1] = ch.v[1];
            }
            cl54_block<R>(c, d + 3 * blk, a, a + 6, s + 6 * blk, acc + 6 * blk);
            // one block's 24 reals in flight at a time (the compiler would otherwise issue
            // all 54 loads at once and hold them in registers)
            asm volatile("" ::: "memory");
        }
    } else {
        R a[NC * T::PER_CHUNK];  // 56 reals
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            Chunk<P> ch = load_chunk<P>(cl, base + (long)k * kSB);
#pragma unroll
            for (int j = 0; j < T::PER_CHUNK; ++j) a[k * T::PER_CHUNK + j] = to_real<P>(ch.v[j]);
        }
        cl54_block<R>(c, a, a + 6, a + 12, s, acc);
        cl54_block<R>(c, a + 3, a + 30, a + 36, s + 6, acc + 6);
    }
}

// the 72 clover reals of site (par, i) into registers
template <int P>
__device__ __forceinline__ void load_clover(const void* clover, int Vh, int par, int i,
                                            typename Traits<P>::real a[72])
{
    using T = Traits<P>;
    const long base = chunk_at(Vh, T::CLOVER_CHUNKS, par, 0, i);
#pragma unroll
    for (int k = 0; k < T::CLOVER_CHUNKS; ++k) {
        Chunk<P> c = load_chunk<P>(clover, base + (long)k * kSB);
#pragma unroll
        for (int j = 0; j < T::PER_CHUNK; ++j) a[k * T::PER_CHUNK + j] = to_real<P>(c.v[j]);
    }
}

}  // namespace qdw
