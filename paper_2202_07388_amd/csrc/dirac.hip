// dirac.hip -- the Wilson-clover operator D and D^+ on eo-SoA fields.
//
// One lane per output site; a 256-lane workgroup owns 128 consecutive even-odd indices
// of BOTH parities (lanes 0..127 even, 128..255 odd). The even site with index i and the
// odd site with index i are lexicographic neighbours along x3, so a workgroup covers a
// compact run of the lattice: the eight links a site reads are mostly the same links its
// neighbours in the workgroup read (every link joins an even and an odd site), and the
// neighbour spinors are shared through L1/L2. Workgroups are mapped XCD-contiguously.
//
// Per hop the neighbour spinor is spin-projected with (1 -+ gamma_mu) to two spin
// components, multiplied by the link (third row rebuilt from the first two, times the
// U(1) phase, boundary sign and the factor -1/2 folded into one complex coefficient)
// and expanded back to four spins. D^+ = gamma_5 D gamma_5 flips the projector signs.
#include "qdw_host.h"

using namespace qdw;

namespace {

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

// link rows 0, 1 (6 complex) and the phase exp(i theta) of link (par, i, mu)
template <int P>
__device__ __forceinline__ void load_link(const void* links, const void* theta, int Vh, int par,
                                          int i, int mu, cx<typename Traits<P>::real> u[6],
                                          cx<typename Traits<P>::real>& ph)
{
    using T = Traits<P>;
    using R = typename T::real;
    const long row = (long)(par * 4 + mu);
    if constexpr (P == F64 || P == F32) {
#pragma unroll
        for (int k = 0; k < T::LINK_CHUNKS; ++k) {
            Chunk<P> c = load_chunk_cached<P>(links, (row * T::LINK_CHUNKS + k) * Vh + i);
#pragma unroll
            for (int j = 0; j < T::PER_CHUNK / 2; ++j)
                u[k * (T::PER_CHUNK / 2) + j] = {c.v[2 * j], c.v[2 * j + 1]};
        }
        const R th = ((const typename T::store*)theta)[row * Vh + i];
        R s, co;
        if constexpr (P == F64) sincos(th, &s, &co);
        else sincosf(th, &s, &co);
        ph = {co, s};
    } else {
        Chunk<P> c0 = load_chunk_cached<P>(links, (row * 2 + 0) * Vh + i);
        Chunk<P> c1 = load_chunk_cached<P>(links, (row * 2 + 1) * Vh + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = {to_real<P>(c0.v[2 * j]), to_real<P>(c0.v[2 * j + 1])};
        u[4] = {to_real<P>(c1.v[0]), to_real<P>(c1.v[1])};
        u[5] = {to_real<P>(c1.v[2]), to_real<P>(c1.v[3])};
        ph = {to_real<P>(c1.v[4]), to_real<P>(c1.v[5])};
    }
}

// w = c * V h (DAGGER: c * V^+ h) for the two spin components of h; V rebuilt from rows
template <typename R, bool DAGGER>
__device__ __forceinline__ void su3_apply(const cx<R> u[6], cx<R> c, const cx<R> h[6], cx<R> w[6])
{
    cx<R> r2[3];
    r2[0] = conj_(u[1] * u[5] - u[2] * u[4]);
    r2[1] = conj_(u[2] * u[3] - u[0] * u[5]);
    r2[2] = conj_(u[0] * u[4] - u[1] * u[3]);
    const cx<R> m[9] = {u[0], u[1], u[2], u[3], u[4], u[5], r2[0], r2[1], r2[2]};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const cx<R> h0 = c * h[3 * a], h1 = c * h[3 * a + 1], h2 = c * h[3 * a + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (!DAGGER) {
                w[3 * a + r] = m[3 * r] * h0 + m[3 * r + 1] * h1 + m[3 * r + 2] * h2;
            } else {
                w[3 * a + r] = cmul_conj(m[r], h0) + cmul_conj(m[3 + r], h1) + cmul_conj(m[6 + r], h2);
            }
        }
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
    constexpr int CPB = T::CLOVER_CHUNKS / 2;  // chunks per block
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        R a[36];
#pragma unroll
        for (int k = 0; k < CPB; ++k) {
            Chunk<P> c = load_chunk<P>(clover, ((long)par * T::CLOVER_CHUNKS + b * CPB + k) * Vh + i);
#pragma unroll
            for (int j = 0; j < T::PER_CHUNK; ++j) a[k * T::PER_CHUNK + j] = to_real<P>(c.v[j]);
        }
        const cx<R>* v = s + 6 * b;
        cx<R> o[6];
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
#pragma unroll
        for (int r = 0; r < 6; ++r) acc[6 * b + r] = o[r];
    }
}

template <int P, int MU, bool DAG>
__device__ __forceinline__ void hop_pair(const Geom& g, const void* in, const void* links,
                                         const void* theta, int par, int i, const int x[4], int lex,
                                         cx<typename Traits<P>::real> acc[12])
{
    using R = typename Traits<P>::real;
    constexpr int SF = DAG ? +1 : -1;  // forward projector 1 + SF gamma
    constexpr int SB = -SF;            // backward projector
    cx<R> s[12], h[6], w[6], u[6], ph;
    // forward: U_mu(x) (1 -+ gamma) psi(x + mu), link owned by x
    {
        const int j = lex_fwd(g, x, lex, MU) >> 1;
        load_spinor<P>(in, g.Vh, 1 - par, j, s);
        project<R, MU, SF>(s, h);
        load_link<P>(links, theta, g.Vh, par, i, MU, u, ph);
        const R sg = (MU == 0 && x[0] == g.L[0] - 1) ? (R)(-0.5 * g.bc_t) : (R)-0.5;
        su3_apply<R, false>(u, scale(ph, sg), h, w);
        expand_add<R, MU, SF>(w, acc);
    }
    // backward: U_mu(x - mu)^+ (1 +- gamma) psi(x - mu), link owned by x - mu
    {
        const int j = lex_bwd(g, x, lex, MU) >> 1;
        load_spinor<P>(in, g.Vh, 1 - par, j, s);
        project<R, MU, SB>(s, h);
        load_link<P>(links, theta, g.Vh, 1 - par, j, MU, u, ph);
        const R sg = (MU == 0 && x[0] == 0) ? (R)(-0.5 * g.bc_t) : (R)-0.5;
        su3_apply<R, true>(u, scale(conj_(ph), sg), h, w);
        expand_add<R, MU, SB>(w, acc);
    }
}

template <int P, bool DAG>
__global__ __launch_bounds__(256) void dw_kernel(Geom g, const void* __restrict__ in,
                                                 void* __restrict__ out,
                                                 const void* __restrict__ links,
                                                 const void* __restrict__ theta,
                                                 const void* __restrict__ clover)
{
    using R = typename Traits<P>::real;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int par = threadIdx.x >> 7;
    const int i = tile * 128 + (threadIdx.x & 127);
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<R> acc[12];
    {
        cx<R> s[12];
        load_spinor<P>(in, g.Vh, par, i, s);
        clover_apply<P>(clover, g.Vh, par, i, s, acc);
    }
    hop_pair<P, 0, DAG>(g, in, links, theta, par, i, x, lex, acc);
    hop_pair<P, 1, DAG>(g, in, links, theta, par, i, x, lex, acc);
    hop_pair<P, 2, DAG>(g, in, links, theta, par, i, x, lex, acc);
    hop_pair<P, 3, DAG>(g, in, links, theta, par, i, x, lex, acc);
    store_spinor<P>(out, g.Vh, par, i, acc);
}

template <int P, bool DAG>
int launch(qdw_op* op, const void* in, void* out, hipStream_t st)
{
    const Geom& g = op->g;
    const int nblk = (g.Vh + 127) / 128;
    dw_kernel<P, DAG><<<nblk, 256, 0, st>>>(g, in, out, op->links[P], op->theta[P], op->clover[P]);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

template <bool DAG>
int dispatch(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_apply: null argument");
    QDW_CHECK(in != out, QDW_EINVAL, "dw_apply: in and out must be distinct fields");
    hipStream_t st = (hipStream_t)stream;
    switch (prec) {
    case QDW_F64: return launch<F64, DAG>(op, in, out, st);
    case QDW_F32: return launch<F32, DAG>(op, in, out, st);
    case QDW_F16S: return launch<F16S, DAG>(op, in, out, st);
    case QDW_BF16S: return launch<BF16S, DAG>(op, in, out, st);
    default: QDW_CHECK(false, QDW_EINVAL, "dw_apply: bad precision");
    }
}

}  // namespace

namespace qdw {
// internal entry used by the solvers (same kernels, no argument re-validation)
int dw_launch(qdw_op* op, const void* in, void* out, int prec, bool dag, hipStream_t st)
{
    if (dag) return dispatch<true>(op, in, out, (qdw_prec)prec, st);
    return dispatch<false>(op, in, out, (qdw_prec)prec, st);
}
}  // namespace qdw

extern "C" int dw_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    return dispatch<false>(op, in, out, prec, stream);
}

extern "C" int dw_dag_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    return dispatch<true>(op, in, out, prec, stream);
}
