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
        const R* dp = (const R*)dets + 2 * (row * Vh + i);
        d = {dp[0], dp[1]};
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
    const cx<R> r2[3] = {d * conj_(u[1] * u[5] - u[2] * u[4]),
                         d * conj_(u[2] * u[3] - u[0] * u[5]),
                         d * conj_(u[0] * u[4] - u[1] * u[3])};
    const cx<R> m[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const cx<R> h0 = h[3 * a], h1 = h[3 * a + 1], h2 = h[3 * a + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (!DAGGER)
                w[3 * a + r] = m[3 * r] * h0 + m[3 * r + 1] * h1 + m[3 * r + 2] * h2;
            else
                w[3 * a + r] = cmul_conj(m[r], h0) + cmul_conj(m[3 + r], h1) + cmul_conj(m[6 + r], h2);
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
            o[r] = o[r] + e * v[q];
            o[q] = o[q] + cmul_conj(e, v[r]);
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
