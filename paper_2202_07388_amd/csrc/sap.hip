// sap.hip -- Schwarz alternating procedure as a preconditioner (paper Sec. 3, Fig. 2
// and 3): the lattice is cut into blocks coloured like a chessboard; one cycle solves
// every block of colour 0, then every block of colour 1, each approximately by nmr
// minimal-residual steps on the block-restricted operator D_b (hops leaving the block
// dropped), with the residual brought up to date between the two colours.
//
// GPU mapping: one workgroup per block, one lane per site (block volume 64..256 sites).
// A block's residual lives in LDS for all nmr steps; every lane keeps its own clover
// blocks and its four forward links in registers. The backward hop into a site is
// computed by the lane that owns the link (the site below it) and handed over through
// LDS as a transported half spinor, so each link is read from HBM once per sweep.
// Storage precision SP (FP32, FP16 or BF16) for every field in HBM; FP32 arithmetic;
// block reductions accumulate per lane in FP32 and combine across lanes in FP64.
//
// After a colour's block solves, the block residuals r_b are exactly the new residual
// on that colour; the other colour's residual loses the hops from the block corrections
// that cross into it (D_partial chi, Fig. 3 right), applied by a second kernel.
#include <map>
#include <mutex>

#include "sap.h"

#include "dirac_core.h"

namespace qdw {

int make_block_geom(const Geom& g, const int bs[4], BlockGeom* B)
{
    int vol = 1;
    for (int mu = 0; mu < 4; ++mu) {
        QDW_CHECK(bs[mu] >= 1 && g.L[mu] % bs[mu] == 0, QDW_EBLOCK,
                  "SAP: block extents must divide the lattice extents");
        const int nb = g.L[mu] / bs[mu];
        QDW_CHECK(nb >= 2 && nb % 2 == 0, QDW_EBLOCK,
                  "SAP: need an even number (>= 2) of blocks in every direction");
        B->bs[mu] = bs[mu];
        B->nb[mu] = nb;
        vol *= bs[mu];
    }
    QDW_CHECK(vol >= 64 && vol <= 256 && vol % 64 == 0, QDW_EBLOCK,
              "SAP: block volume must be 64, 128, 192 or 256 sites");
    B->bvol = vol;
    B->lstride[3] = 1;
    B->lstride[2] = bs[3];
    B->lstride[1] = bs[3] * bs[2];
    B->lstride[0] = bs[3] * bs[2] * bs[1];
    B->nblk = B->nb[0] * B->nb[1] * B->nb[2] * B->nb[3];
    return QDW_OK;
}

namespace {

constexpr int kBMax = 256;

template <int SP, int MU>
__device__ __forceinline__ void push_backward(float (*hb)[12][kBMax], const BlockGeom& B,
                                              const int l[4], int t, const cx<float> r[12],
                                              const cx<float> u[6], cx<float> d)
{
    if (l[MU] < B.bs[MU] - 1) {
        cx<float> h[6], w[6];
        project<float, MU, +1>(r, h);
        su3_mul<float, true>(u, d, h, w);
        const int dst = t + B.lstride[MU];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            hb[MU][2 * c][dst] = w[c].re;
            hb[MU][2 * c + 1][dst] = w[c].im;
        }
    }
}

template <int SP, int MU>
__device__ __forceinline__ void hop_forward(float (*rl)[kBMax], const BlockGeom& B, const int l[4],
                                            int t, const cx<float> u[6], cx<float> d,
                                            cx<float> v[12])
{
    if (l[MU] < B.bs[MU] - 1) {
        const int src = t + B.lstride[MU];
        cx<float> s[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) s[c] = {rl[2 * c][src], rl[2 * c + 1][src]};
        project<float, MU, -1>(s, h);
        su3_mul<float, false>(u, d, h, w);
        expand_add<float, MU, -1>(w, v);
    }
}

template <int MU, int N = kBMax>
__device__ __forceinline__ void hop_backward(float (*hb)[12][N], const int l[4], int t,
                                             cx<float> v[12])
{
    if (l[MU] > 0) {
        cx<float> w[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) w[c] = {hb[MU][2 * c][t], hb[MU][2 * c + 1][t]};
        expand_add<float, MU, +1>(w, v);
    }
}

// The lane's clover blocks (or their inverses) and its four forward links, held in
// registers through all MR steps of a block: as FP32 values for FP32 storage, and as the
// stored 16-bit values for FP16 / BF16 storage (half the registers, which lets two
// workgroups share a CU), widened to FP32 where they are used (exactly). opaque() hides the
// stored values from the optimiser, so that the widening is redone after each call rather
// than hoisted out of the loop into registers held for the whole kernel.
template <int SP, bool PACKED = (SP == F16S || SP == BF16S)>
struct SiteOps {
    float cl[72];
    cx<float> u[4][6], d[4];
    __device__ __forceinline__ void load(const Geom& g, const void* clover, const void* links,
                                         const void* dets, int par, int i)
    {
        load_clover<SP>(clover, g.Vh, par, i, cl);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) load_link<SP>(links, dets, g.Vh, par, i, mu, u[mu], d[mu]);
    }
    __device__ __forceinline__ void opaque() {}
    template <int MU>
    __device__ __forceinline__ void link(cx<float> uu[6], cx<float>& dd) const
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) uu[c] = u[MU][c];
        dd = d[MU];
    }
    // o = A v (both chirality blocks)
    __device__ __forceinline__ void diag(const cx<float> v[12], cx<float> o[12]) const
    {
        herm6_apply<float>(cl, v, o);
        herm6_apply<float>(cl + 36, v + 6, o + 6);
    }
};

template <int SP>
struct SiteOps<SP, true> {
    uint32_t cl[36];    // the 72 stored 16-bit clover values, two per register
    uint32_t lk[4][7];  // per link: rows 0, 1 (12 values) and det U (2 values)
    __device__ __forceinline__ static float widen(uint32_t w, int hi)
    {
        const uint16_t b = hi ? (uint16_t)(w >> 16) : (uint16_t)(w & 0xFFFFu);
        if constexpr (SP == F16S) {
            _Float16 h;
            __builtin_memcpy(&h, &b, 2);
            return (float)h;
        } else {
            return bf16_to_float(b);
        }
    }
    __device__ __forceinline__ void load(const Geom& g, const void* clover, const void* links,
                                         const void* dets, int par, int i)
    {
        const long base = chunk_at(g.Vh, Traits<SP>::CLOVER_CHUNKS, par, 0, i);
#pragma unroll
        for (int k = 0; k < Traits<SP>::CLOVER_CHUNKS; ++k) {
            const Chunk<SP> c = load_chunk<SP>(clover, base + (long)k * kSB);
            __builtin_memcpy(cl + 4 * k, &c, 16);
        }
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const long row = (long)(par * 4 + mu);
            const Chunk<SP> c0 = load_chunk_cached<SP>(links, chunk_at(g.Vh, 2, row, 0, i));
            const Chunk<SP> c1 = load_chunk_cached<SP>(links, chunk_at(g.Vh, 2, row, 1, i));
            uint32_t w1[4];
            __builtin_memcpy(lk[mu], &c0, 16);
            __builtin_memcpy(w1, &c1, 16);
            lk[mu][4] = w1[0];
            lk[mu][5] = w1[1];
            lk[mu][6] = w1[2];
        }
        (void)dets;
    }
    __device__ __forceinline__ void opaque()
    {
#pragma unroll
        for (int k = 0; k < 36; ++k) asm volatile("" : "+v"(cl[k]));
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int k = 0; k < 7; ++k) asm volatile("" : "+v"(lk[mu][k]));
    }
    template <int MU>
    __device__ __forceinline__ void link(cx<float> uu[6], cx<float>& dd) const
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) uu[c] = {widen(lk[MU][c], 0), widen(lk[MU][c], 1)};
        dd = {widen(lk[MU][6], 0), widen(lk[MU][6], 1)};
    }
    __device__ __forceinline__ void diag(const cx<float> v[12], cx<float> o[12]) const
    {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            float a[36];
#pragma unroll
            for (int k = 0; k < 36; ++k) a[k] = widen(cl[(36 * b + k) >> 1], (36 * b + k) & 1);
            herm6_apply<float>(a, v + 6 * b, o + 6 * b);
        }
    }
};

// w = M h (DAGGER: M^+ h) with the full 3x3 matrix M, for both spin components of h
template <bool DAGGER>
__device__ __forceinline__ void mat_mul(const cx<float> m[9], const cx<float> h[6], cx<float> w[6])
{
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const cx<float> h0 = h[3 * a], h1 = h[3 * a + 1], h2 = h[3 * a + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            if (!DAGGER)
                w[3 * a + r] = cmadd(cmadd(m[3 * r] * h0, m[3 * r + 1], h1), m[3 * r + 2], h2);
            else
                w[3 * a + r] = cmadd_conj(cmadd_conj(cmul_conj(m[r], h0), m[3 + r], h1), m[6 + r], h2);
        }
    }
}

// direction MU of a block-D application for this lane: the hand-over of U^+ (1 + gamma) r
// to the +MU neighbour (read by it after the barrier) and the forward hop from it, with the
// link widened and its third row rebuilt once for both
template <int SP, int MU>
__device__ __forceinline__ void push_and_forward(float (*hb)[12][kBMax], float (*rl)[kBMax],
                                                 const BlockGeom& B, const int l[4], int t,
                                                 const cx<float> r[12], const SiteOps<SP>& so,
                                                 cx<float> v[12])
{
    if (l[MU] < B.bs[MU] - 1) {
        cx<float> u[6], d, m[9];
        so.template link<MU>(u, d);
        m[6] = d * conj_(cmadd(u[1] * u[5], -u[2], u[4]));
        m[7] = d * conj_(cmadd(u[2] * u[3], -u[0], u[5]));
        m[8] = d * conj_(cmadd(u[0] * u[4], -u[1], u[3]));
#pragma unroll
        for (int c = 0; c < 6; ++c) m[c] = u[c];
        const int nb = t + B.lstride[MU];
        cx<float> h[6], w[6];
        project<float, MU, +1>(r, h);
        mat_mul<true>(m, h, w);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            hb[MU][2 * c][nb] = w[c].re;
            hb[MU][2 * c + 1][nb] = w[c].im;
        }
        cx<float> sn[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) sn[c] = {rl[2 * c][nb], rl[2 * c + 1][nb]};
        project<float, MU, -1>(sn, h);
        mat_mul<false>(m, h, w);
        expand_add<float, MU, -1>(w, v);
    }
}

// The same hand-over and forward hop with the neighbour's lane given explicitly (-1: the
// neighbour is outside the block), for blocks whose lanes are not numbered by site
template <int SP, int MU, int N>
__device__ __forceinline__ void push_to(float (*hb)[12][N], int dst, const cx<float> r[12],
                                        const cx<float> u[6], cx<float> d)
{
    if (dst >= 0) {
        cx<float> h[6], w[6];
        project<float, MU, +1>(r, h);
        su3_mul<float, true>(u, d, h, w);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            hb[MU][2 * c][dst] = w[c].re;
            hb[MU][2 * c + 1][dst] = w[c].im;
        }
    }
}

template <int SP, int MU, int N>
__device__ __forceinline__ void forward_from(float (*rl)[N], int src, const cx<float> u[6],
                                             cx<float> d, cx<float> v[12])
{
    if (src >= 0) {
        cx<float> s[12], h[6], w[6];
#pragma unroll
        for (int c = 0; c < 12; ++c) s[c] = {rl[2 * c][src], rl[2 * c + 1][src]};
        project<float, MU, -1>(s, h);
        su3_mul<float, false>(u, d, h, w);
        expand_add<float, MU, -1>(w, v);
    }
}

// sum over the block of a per-lane value (one FP64 result, the same in every lane);
// `slots` must not be read by any lane between the barrier inside and the next barrier
__device__ __forceinline__ double block_sum(double v, double* slots, int t, int nw)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((t & 63) == 0) slots[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += slots[w];
    return s;
}

// acc += the hops of D delta that enter x's block from outside (without the -1/2), for
// a site x of a block of colour 1 - `colour` (delta lives on the colour blocks)
template <int SP, int MU>
__device__ __forceinline__ void cross_hops(const Geom& g, const BlockGeom& B, const void* delta,
                                           const void* links, const void* dets, int par, int i,
                                           const int x[4], int lex, cx<float> acc[12], bool& any)
{
    cx<float> s[12], h[6], w[6], u[6], d;
    if (x[MU] % B.bs[MU] == B.bs[MU] - 1) {
        const int j = lex_fwd(g, x, lex, MU) >> 1;
        load_spinor<SP>(delta, g.Vh, 1 - par, j, s);
        project<float, MU, -1>(s, h);
        if (MU == 0 && g.bc_t < 0 && x[0] == g.L[0] - 1)
            for (int c = 0; c < 6; ++c) h[c] = {-h[c].re, -h[c].im};
        load_link<SP>(links, dets, g.Vh, par, i, MU, u, d);
        su3_mul<float, false>(u, d, h, w);
        expand_add<float, MU, -1>(w, acc);
        any = true;
    }
    if (x[MU] % B.bs[MU] == 0) {
        const int j = lex_bwd(g, x, lex, MU) >> 1;
        load_spinor<SP>(delta, g.Vh, 1 - par, j, s);
        project<float, MU, +1>(s, h);
        if (MU == 0 && g.bc_t < 0 && x[0] == 0)
            for (int c = 0; c < 6; ++c) h[c] = {-h[c].re, -h[c].im};
        load_link<SP>(links, dets, g.Vh, 1 - par, j, MU, u, d);
        su3_mul<float, true>(u, d, h, w);
        expand_add<float, MU, +1>(w, acc);
        any = true;
    }
}

// r(x) -= (D delta)(x) over the hops that enter x's block from outside, applied to the
// block residual as a block kernel loads it (delta: the corrections of the other colour's
// blocks, from the launch before; nullptr: nothing to apply). This is the residual update
// between the two colours (Fig. 3 right) done by the receiving blocks, in FP32 on the loaded
// values, instead of a separate pass over the lattice (sap_boundary_kernel) that rounds r
// to storage once more.
template <int SP>
__device__ __forceinline__ void apply_cross_hops(const Geom& g, const BlockGeom& B, const void* delta,
                                                 const void* links, const void* dets, int par,
                                                 int i, const int x[4], int lex, cx<float> r[12])
{
    if (!delta) return;
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
    bool any = false;
    cross_hops<SP, 0>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 1>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 2>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 3>(g, B, delta, links, dets, par, i, x, lex, acc, any);
#pragma unroll
    for (int c = 0; c < 12; ++c) r[c] = r[c] + scale(acc[c], 0.5f);  // hops carry -1/2
}

// 16-bit storage: registers for two waves per SIMD (two 256-site blocks per CU)
template <int SP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SP == F32 ? 1 : 2)))
void sap_mr_kernel(Geom g, BlockGeom B, int colour, int nmr,
                                                     void* __restrict__ rs, void* __restrict__ psis,
                                                     void* __restrict__ delta,
                                                     const void* __restrict__ links,
                                                     const void* __restrict__ dets,
                                                     const void* __restrict__ clover,
                                                     RhsStride bat, SapAdapt ad)
{
    __shared__ float rl[24][kBMax];
    __shared__ float hb[4][12][kBMax];
    __shared__ double red[4][3];
    __shared__ double red2[2][4];
    // right-hand side `rhs` of a batch (fields at a fixed byte stride), block `blk` of the
    // colour
    const int rhs = (int)blockIdx.x % bat.nrhs, blk = (int)blockIdx.x / bat.nrhs;
    if (bat.gate && !bat.gate[(long)rhs * bat.gstride]) return;
    rs = (char*)rs + rhs * bat.fstride;
    psis = (char*)psis + rhs * bat.fstride;
    delta = (char*)delta + rhs * bat.fstride;
    const int t = threadIdx.x;
    const int nw = B.bvol >> 6;
    // the blockIdx-th block of this colour (blocks per x3 row is even, so colours alternate)
    int b[4];
    {
        int r = 2 * blk;
        b[3] = r % B.nb[3]; r /= B.nb[3];
        b[2] = r % B.nb[2]; r /= B.nb[2];
        b[1] = r % B.nb[1];
        b[0] = r / B.nb[1];
        if (((b[0] + b[1] + b[2] + b[3]) & 1) != colour) b[3] += 1;
    }
    int l[4];
    {
        int r = t;
        l[3] = r % B.bs[3]; r /= B.bs[3];
        l[2] = r % B.bs[2]; r /= B.bs[2];
        l[1] = r % B.bs[1];
        l[0] = r / B.bs[1];
    }
    int x[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) x[mu] = b[mu] * B.bs[mu] + l[mu];
    const int lex = ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
    const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int i = lex >> 1;

    cx<float> r[12], chi[12];
    load_spinor<SP>(rs, g.Vh, par, i, r);
    SiteOps<SP> so;
    so.load(g, clover, links, dets, par, i);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        chi[c] = {0.f, 0.f};
        rl[2 * c][t] = r[c].re;
        rl[2 * c + 1][t] = r[c].im;
    }
    // adaptive exits (Sec. 3.2): the block residual norm before the first step and after
    // every step decides, uniformly in the workgroup, whether the MR loop goes on
    double prev = 0.0;
    int nsteps = 0;
    bool go = true;
    if (ad.on) {
        float l2 = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) l2 += r[c].re * r[c].re + r[c].im * r[c].im;
        prev = sqrt(block_sum((double)l2, red2[0], t, nw));
        go = !(prev < (double)ad.tol);
    }
    for (int k = 0; k < nmr && go; ++k) {
        __syncthreads();  // rl holds the current block residual
        cx<float> v[12], vh[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) vh[c] = {0.f, 0.f};
        so.opaque();
        push_and_forward<SP, 0>(hb, rl, B, l, t, r, so, vh);
        push_and_forward<SP, 1>(hb, rl, B, l, t, r, so, vh);
        push_and_forward<SP, 2>(hb, rl, B, l, t, r, so, vh);
        push_and_forward<SP, 3>(hb, rl, B, l, t, r, so, vh);
        __syncthreads();  // every pushed half spinor is in hb
        hop_backward<0>(hb, l, t, vh);
        hop_backward<1>(hb, l, t, vh);
        hop_backward<2>(hb, l, t, vh);
        hop_backward<3>(hb, l, t, vh);
        // v = D_b r = A r - 1/2 (hops inside the block)
        so.opaque();
        so.diag(r, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = v[c] - scale(vh[c], 0.5f);
        // omega = (v, r) / (v, v) over the block
        float nre = 0.f, nim = 0.f, den = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cx<float> z = cmadd_conj(cx<float>{nre, nim}, v[c], r[c]);
            nre = z.re;
            nim = z.im;
            den = fmar(v[c].re, v[c].re, fmar(v[c].im, v[c].im, den));
        }
        double a0 = nre, a1 = nim, a2 = den;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
            a2 += __shfl_xor(a2, o, 64);
        }
        if ((t & 63) == 0) {
            red[t >> 6][0] = a0;
            red[t >> 6][1] = a1;
            red[t >> 6][2] = a2;
        }
        __syncthreads();
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int w = 0; w < nw; ++w) {
            s0 += red[w][0];
            s1 += red[w][1];
            s2 += red[w][2];
        }
        const cx<float> om = s2 > 0.0 ? cx<float>{(float)(s0 / s2), (float)(s1 / s2)}
                                      : cx<float>{0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            chi[c] = chi[c] + om * r[c];
            r[c] = r[c] - om * v[c];
        }
        if (ad.on) {
            float l2 = 0.f;
#pragma unroll
            for (int c = 0; c < 12; ++c) l2 += r[c].re * r[c].re + r[c].im * r[c].im;
            double v2 = l2;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v2 += __shfl_xor(v2, o, 64);
            if ((t & 63) == 0) red2[(k + 1) & 1][t >> 6] = v2;
        }
        __syncthreads();  // all lanes have read red and rl of this step
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            rl[2 * c][t] = r[c].re;
            rl[2 * c + 1][t] = r[c].im;
        }
        ++nsteps;
        if (ad.on) {
            double c2 = 0.0;
            for (int w = 0; w < nw; ++w) c2 += red2[(k + 1) & 1][w];
            const double cur = sqrt(c2);
            if ((nsteps >= 4 && cur > (double)ad.alpha * prev) || cur > prev ||
                cur < (double)ad.tol)
                go = false;
            else
                prev = cur;
        }
    }
    if (ad.steps && t == 0) ad.steps[blk] = nsteps;
    cx<float> p[12];
    load_spinor<SP>(psis, g.Vh, par, i, p);
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = p[c] + chi[c];
    store_spinor<SP>(psis, g.Vh, par, i, p);
    store_spinor<SP>(delta, g.Vh, par, i, chi);
    store_spinor<SP>(rs, g.Vh, par, i, r);
}

// The same block solve through the block's even-odd reduction: for the block residual
// r = (r_e, r_o) (A = the clover term, H = the sum of the hops inside the block, so that
// D_eo = D_oe = -1/2 H between the parities)
//   r^_e  = r_e - D_eo A_oo^-1 r_o = r_e + 1/2 H A_oo^-1 r_o
//   chi_e = nmr MR steps from 0 on D^_b = A_ee - 1/4 H A_oo^-1 H with source r^_e
//   chi_o = A_oo^-1 (r_o - D_oe chi_e) = A_oo^-1 (r_o + 1/2 H chi_e)
// after which the block residual is (the MR residual, 0). Even lanes hold A, odd lanes
// A^-1 in registers; every application of H is one pass of the in-block hops over LDS.
template <int SP, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SP == F32 ? 1 : 2)))
void sap_mr_eo_kernel(Geom g, BlockGeom B, int colour, int nmr,
                                                        void* __restrict__ rs,
                                                        void* __restrict__ psis,
                                                        void* __restrict__ delta,
                                                        const void* __restrict__ links,
                                                        const void* __restrict__ dets,
                                                        const void* __restrict__ clover,
                                                        const void* __restrict__ cloverinv,
                                                        RhsStride bat, const void* odelta)
{
    // Hand-over buffers. Lanes numbered by parity (SPLIT, below): a hop pass writes rl only
    // from its sending half and hb only for its receiving half, so both are indexed by the
    // lane's place within its half and take half the room; that pays for two sets used in
    // turn, and a pass then needs no barrier at its end (the set it wrote is next written
    // two passes later, after both barriers of the pass between). Lanes numbered by site:
    // one full-size set and a third barrier per pass.
    constexpr int NB = SPLIT ? 2 : 1, NL = SPLIT ? kBMax / 2 : kBMax;
    __shared__ float rl[NB][24][NL];
    __shared__ float hb[NB][4][12][NL];
    __shared__ double red[4][3];
    const int rhs = (int)blockIdx.x % bat.nrhs, blk = (int)blockIdx.x / bat.nrhs;
    if (bat.gate && !bat.gate[(long)rhs * bat.gstride]) return;
    rs = (char*)rs + rhs * bat.fstride;
    psis = (char*)psis + rhs * bat.fstride;
    delta = (char*)delta + rhs * bat.fstride;
    if (odelta) odelta = (const char*)odelta + rhs * bat.fstride;
    const int t = threadIdx.x;
    const int nw = B.bvol >> 6;
    int b[4];
    {
        int r = 2 * blk;
        b[3] = r % B.nb[3]; r /= B.nb[3];
        b[2] = r % B.nb[2]; r /= B.nb[2];
        b[1] = r % B.nb[1];
        b[0] = r / B.nb[1];
        if (((b[0] + b[1] + b[2] + b[3]) & 1) != colour) b[3] += 1;
    }
    // Lanes by parity: with an even x3 extent the block's sites 2e and 2e + 1 (its local
    // index) have opposite parities, and lane e (first half) takes the even one of the
    // pair, lane half + e the odd one. Every hop pass below sends from one parity to the
    // other, so whole wavefronts skip the half they have no part in. With an odd x3
    // extent lanes are numbered by site (correct, without the saving).
    const int half = B.bvol >> 1;
    constexpr bool split = SPLIT;  // launched so only for an even x3 block extent
    const int bpar = (b[0] * B.bs[0] + b[1] * B.bs[1] + b[2] * B.bs[2] + b[3] * B.bs[3]) & 1;
    auto local = [&](int site, int lc[4]) {
        int r = site;
        lc[3] = r % B.bs[3]; r /= B.bs[3];
        lc[2] = r % B.bs[2]; r /= B.bs[2];
        lc[1] = r % B.bs[1];
        lc[0] = r / B.bs[1];
    };
    int site = t;
    if (split) {
        const int want = t >= half ? 1 : 0;
        const int s0 = 2 * (t - want * half);
        int l0[4];
        local(s0, l0);
        site = s0 + (((bpar + l0[0] + l0[1] + l0[2] + l0[3]) & 1) != want ? 1 : 0);
    }
    int l[4];
    local(site, l);
    int x[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) x[mu] = b[mu] * B.bs[mu] + l[mu];
    const int lex = ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
    const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int i = lex >> 1;
    const bool ev = par == 0;
    // places in the hand-over buffers of the +mu neighbours inside the block (the other
    // parity; with SPLIT, within that parity's half), -1 at the block edge, and of this lane
    int nbl[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int sn = site + B.lstride[mu];
        nbl[mu] = l[mu] < B.bs[mu] - 1 ? (split ? (sn >> 1) : sn) : -1;
    }
    const int tl = split ? t - par * half : t;
    int set = 0;  // hand-over set of the next pass (SPLIT: alternating)

    cx<float> r[12];
    load_spinor<SP>(rs, g.Vh, par, i, r);
    apply_cross_hops<SP>(g, B, odelta, links, dets, par, i, x, lex, r);
    SiteOps<SP> so;  // A on even sites, A^-1 on odd sites
    so.load(g, ev ? clover : cloverinv, links, dets, par, i);

    auto diag = [&](const cx<float> v[12], cx<float> o[12]) {
        so.opaque();
        so.diag(v, o);
    };
    // vh = H src on the lanes of the parity other than `from` (0 on the lanes of `from`);
    // src is non-zero on the lanes of `from` only
    auto hops = [&](int from, const cx<float> src[12], cx<float> vh[12]) {
        const bool sends = par == from;
        float (*rb)[NL] = rl[set];
        float (*hbb)[12][NL] = hb[set];
        if (SPLIT) set ^= 1;
        if (sends) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                rb[2 * c][tl] = src[c].re;
                rb[2 * c + 1][tl] = src[c].im;
            }
        }
        __syncthreads();  // rl holds src
#pragma unroll
        for (int c = 0; c < 12; ++c) vh[c] = {0.f, 0.f};
        cx<float> u[6], d;
        so.opaque();
        if (sends) {
            so.template link<0>(u, d);
            push_to<SP, 0, NL>(hbb, nbl[0], src, u, d);
            so.template link<1>(u, d);
            push_to<SP, 1, NL>(hbb, nbl[1], src, u, d);
            so.template link<2>(u, d);
            push_to<SP, 2, NL>(hbb, nbl[2], src, u, d);
            so.template link<3>(u, d);
            push_to<SP, 3, NL>(hbb, nbl[3], src, u, d);
        } else {
            so.template link<0>(u, d);
            forward_from<SP, 0, NL>(rb, nbl[0], u, d, vh);
            so.template link<1>(u, d);
            forward_from<SP, 1, NL>(rb, nbl[1], u, d, vh);
            so.template link<2>(u, d);
            forward_from<SP, 2, NL>(rb, nbl[2], u, d, vh);
            so.template link<3>(u, d);
            forward_from<SP, 3, NL>(rb, nbl[3], u, d, vh);
        }
        __syncthreads();  // every pushed half spinor is in hb
        if (!sends) {
            hop_backward<0, NL>(hbb, l, tl, vh);
            hop_backward<1, NL>(hbb, l, tl, vh);
            hop_backward<2, NL>(hbb, l, tl, vh);
            hop_backward<3, NL>(hbb, l, tl, vh);
        }
        if (!SPLIT) __syncthreads();  // rl and hb are free again
    };
    const cx<float> z = {0.f, 0.f};
    cx<float> w[12], vh[12], res[12], chi[12];
    // (1) the reduced source
    if (ev) {
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = z;
    } else {
        diag(r, w);
    }
    hops(1, w, vh);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        res[c] = ev ? r[c] + scale(vh[c], 0.5f) : z;
        chi[c] = z;
    }
    // (2) MR on the reduced block operator
    for (int k = 0; k < nmr; ++k) {
        hops(0, res, vh);  // odd lanes: H res
        if (ev) {
#pragma unroll
            for (int c = 0; c < 12; ++c) w[c] = z;
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) vh[c] = scale(vh[c], -0.5f);
            diag(vh, w);  // A^-1 D_oe res
        }
        hops(1, w, vh);  // even lanes: H A^-1 D_oe res
        cx<float> v[12];
        if (ev) {
            diag(res, v);
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = v[c] + scale(vh[c], 0.5f);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = z;
        }
        float nre = 0.f, nim = 0.f, den = 0.f;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cx<float> q = cmadd_conj(cx<float>{nre, nim}, v[c], res[c]);
            nre = q.re;
            nim = q.im;
            den = fmar(v[c].re, v[c].re, fmar(v[c].im, v[c].im, den));
        }
        double a0 = nre, a1 = nim, a2 = den;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
            a2 += __shfl_xor(a2, o, 64);
        }
        if ((t & 63) == 0) {
            red[t >> 6][0] = a0;
            red[t >> 6][1] = a1;
            red[t >> 6][2] = a2;
        }
        __syncthreads();
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < nw; ++q) {
            s0 += red[q][0];
            s1 += red[q][1];
            s2 += red[q][2];
        }
        const cx<float> om = s2 > 0.0 ? cx<float>{(float)(s0 / s2), (float)(s1 / s2)}
                                      : cx<float>{0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            chi[c] = chi[c] + om * res[c];
            res[c] = res[c] - om * v[c];
        }
        // red is rewritten only after the two barriers of the next step's first hops
    }
    // (3) the odd half of the block solution
    hops(0, chi, vh);  // odd lanes: H chi_e
    if (!ev) {
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = r[c] + scale(vh[c], 0.5f);
        diag(w, chi);
    }
    // (4) accumulate; the block residual is (res_e, 0)
    cx<float> p[12];
    load_spinor<SP>(psis, g.Vh, par, i, p);
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = p[c] + chi[c];
    store_spinor<SP>(psis, g.Vh, par, i, p);
    store_spinor<SP>(delta, g.Vh, par, i, chi);
    store_spinor<SP>(rs, g.Vh, par, i, res);
}

// r(x) -= (D delta)(x) over the hops that enter x's block from outside
template <int SP>
__global__ __launch_bounds__(256) void sap_boundary_kernel(Geom g, BlockGeom B, int colour,
                                                           void* __restrict__ rs,
                                                           const void* __restrict__ delta,
                                                           const void* __restrict__ links,
                                                           const void* __restrict__ dets,
                                                           RhsStride bat)
{
    const int logical = xcd_tile(blockIdx.x, gridDim.x);
    const int rhs = logical % bat.nrhs, tile = logical / bat.nrhs;
    if (bat.gate && !bat.gate[(long)rhs * bat.gstride]) return;
    rs = (char*)rs + rhs * bat.fstride;
    delta = (const char*)delta + rhs * bat.fstride;
    int par, i;
    if (!walk_site(g, tile, threadIdx.x, par, i)) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const int bc = (x[0] / B.bs[0] + x[1] / B.bs[1] + x[2] / B.bs[2] + x[3] / B.bs[3]) & 1;
    if (bc == colour) return;
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
    bool any = false;
    cross_hops<SP, 0>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 1>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 2>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    cross_hops<SP, 3>(g, B, delta, links, dets, par, i, x, lex, acc, any);
    if (!any) return;
    cx<float> r[12];
    load_spinor<SP>(rs, g.Vh, par, i, r);
#pragma unroll
    for (int c = 0; c < 12; ++c) r[c] = r[c] + scale(acc[c], 0.5f);  // hops carry -1/2
    store_spinor<SP>(rs, g.Vh, par, i, r);
}

template <int SP>
int cycles_impl(qdw_op* op, const BlockGeom& B, int ncy, int nmr, void* rs, void* psis,
                void* delta, const RhsStride& bat_in, int nrhs, bool eo, hipStream_t st)
{
    const Geom& g = op->g;
    RhsStride bat = bat_in;
    bat.nrhs = nrhs;
    const dim3 gmr(B.nblk / 2 * nrhs), gbd(walk_blocks(g) * nrhs);
    for (int cy = 0; cy < ncy; ++cy)
        for (int c = 0; c < 2; ++c) {
            if (eo) {
                // the reduced block solve takes the hops of the other colour's last
                // corrections into its residual as it loads it (cheaper there than a pass
                // of its own: 191 against 168 + 33 us per colour at 24^3 x 48, FP16); after
                // the last colour of the last cycle the residual is not used (only psi is),
                // so that last update is not made
                const void* od = cy == 0 && c == 0 ? nullptr : delta;
                if (B.bs[3] % 2 == 0)
                    sap_mr_eo_kernel<SP, true><<<gmr, B.bvol, 0, st>>>(
                        g, B, c, nmr, rs, psis, delta, op->links[SP], op->det[SP], op->clover[SP],
                        op->cloverinv[SP], bat, od);
                else
                    sap_mr_eo_kernel<SP, false><<<gmr, B.bvol, 0, st>>>(
                        g, B, c, nmr, rs, psis, delta, op->links[SP], op->det[SP], op->clover[SP],
                        op->cloverinv[SP], bat, od);
                QDW_LAUNCH_CHECK();
                continue;
            }
            // the plain block solve, at two waves per SIMD, hides the latency of those
            // loads worse than a pass of their own (169 against 132 + 33 us)
            sap_mr_kernel<SP><<<gmr, B.bvol, 0, st>>>(g, B, c, nmr, rs, psis, delta,
                                                      op->links[SP], op->det[SP],
                                                      op->clover[SP], bat, SapAdapt{});
            QDW_LAUNCH_CHECK();
            sap_boundary_kernel<SP><<<gbd, 2 * g.ts, 0, st>>>(g, B, c, rs, delta, op->links[SP],
                                                              op->det[SP], bat);
            QDW_LAUNCH_CHECK();
        }
    return QDW_OK;
}

template <int SP>
int sap_impl(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy, int nmr,
             const BlockGeom& B, char* work, bool eo, hipStream_t st)
{
    const Geom& g = op->g;
    const size_t fb = spinor_bytes(g, SP);
    void* rs = work;
    void* psis = work + fb;
    void* delta = work + 2 * fb;
    int rc;
    if (ncy == 0 || !(rho_norm > 0.0)) {
        // no preconditioning (the (0, 0) setting), or nothing to precondition
        return run_map(op, Axpby<F64, F64>{rho, phi, ncy == 0 ? 1.0 : 0.0, 0.0, g.Vh}, st);
    }
    const double s = std::sqrt(24.0 * g.V) / rho_norm;
    if ((rc = run_map(op, ScaleNorm<F64, SP>{rho, rs, s, g.Vh}, st, op->scalars + S_SAP))) return rc;
    if ((rc = run_map(op, Zero<SP>{psis, g.Vh}, st))) return rc;
    if ((rc = sap_cycles(op, B, SP, ncy, nmr, rs, psis, delta, RhsStride{}, 1, st, eo))) return rc;
    return run_map(op, Axpby<SP, F64>{psis, phi, 1.0 / s, 0.0, g.Vh}, st);
}

// adaptive cycles: ctrl = {go, cycles done, cycles done over all applications}
__global__ void sap_ctrl_init_kernel(int* ctrl, int reset_total)
{
    ctrl[0] = 1;
    ctrl[1] = 0;
    if (reset_total) ctrl[2] = 0;
}

// after a cycle: count it; go on only while the cycle lowered |r| (sc[S_SAP] holds |r|^2
// before the cycle, sc[S_SAP_NEW] after it)
__global__ void sap_ctrl_cycle_kernel(int* ctrl, double* sc)
{
    if (!ctrl[0]) return;
    ctrl[1] += 1;
    ctrl[2] += 1;
    if (!(sc[S_SAP_NEW] < sc[S_SAP])) ctrl[0] = 0;
    else sc[S_SAP] = sc[S_SAP_NEW];
}

template <int SP>
int adaptive_impl(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy_max,
                  int nmr_max, double alpha, double tol, const BlockGeom& B, char* work,
                  int* steps, hipStream_t st)
{
    const Geom& g = op->g;
    const size_t fb = spinor_bytes(g, SP);
    void* rs = work;
    void* psis = work + fb;
    void* delta = work + 2 * fb;
    int* ctrl = (int*)(work + 3 * fb);
    int rc;
    if (ncy_max == 0 || !(rho_norm > 0.0))
        return run_map(op, Axpby<F64, F64>{rho, phi, ncy_max == 0 ? 1.0 : 0.0, 0.0, g.Vh}, st);
    const double s = std::sqrt(24.0 * g.V) / rho_norm;
    if ((rc = run_map(op, ScaleNorm<F64, SP>{rho, rs, s, g.Vh}, st, op->scalars + S_SAP))) return rc;
    if ((rc = run_map(op, Zero<SP>{psis, g.Vh}, st))) return rc;
    sap_ctrl_init_kernel<<<1, 1, 0, st>>>(ctrl, 0);
    QDW_LAUNCH_CHECK();
    RhsStride gate;
    gate.gate = ctrl;  // every kernel of a cycle returns at once after the stop
    SapAdapt ad;
    ad.alpha = (float)alpha;
    ad.tol = (float)(tol * s);
    ad.on = 1;
    const dim3 gmr(B.nblk / 2, 1), gbd(walk_blocks(g), 1);
    for (int cy = 0; cy < ncy_max; ++cy) {
        for (int c = 0; c < 2; ++c) {
            ad.steps = steps ? steps + (long)(2 * cy + c) * (B.nblk / 2) : nullptr;
            sap_mr_kernel<SP><<<gmr, B.bvol, 0, st>>>(g, B, c, nmr_max, rs, psis, delta,
                                                      op->links[SP], op->det[SP], op->clover[SP],
                                                      gate, ad);
            QDW_LAUNCH_CHECK();
            sap_boundary_kernel<SP><<<gbd, 2 * g.ts, 0, st>>>(g, B, c, rs, delta, op->links[SP],
                                                              op->det[SP], gate);
            QDW_LAUNCH_CHECK();
        }
        if ((rc = run_map(op, Norm2<SP>{rs, g.Vh}, st, op->scalars + S_SAP_NEW))) return rc;
        sap_ctrl_cycle_kernel<<<1, 1, 0, st>>>(ctrl, op->scalars);
        QDW_LAUNCH_CHECK();
    }
    return run_map(op, Axpby<SP, F64>{psis, phi, 1.0 / s, 0.0, g.Vh}, st);
}

}  // namespace

int sap_adaptive_run(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy_max,
                     int nmr_max, double alpha, double tol, const BlockGeom& B, int sdtype,
                     char* work, int* steps, hipStream_t st)
{
    switch (sdtype) {
    case F32: return adaptive_impl<F32>(op, rho, phi, rho_norm, ncy_max, nmr_max, alpha, tol, B, work, steps, st);
    case F16S: return adaptive_impl<F16S>(op, rho, phi, rho_norm, ncy_max, nmr_max, alpha, tol, B, work, steps, st);
    case BF16S: return adaptive_impl<BF16S>(op, rho, phi, rho_norm, ncy_max, nmr_max, alpha, tol, B, work, steps, st);
    default: QDW_CHECK(false, QDW_EINVAL, "SAP: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    }
}

int* sap_ctrl(const qdw_op* op, int sdtype, char* work)
{
    return (int*)(work + 3 * spinor_bytes(op->g, sdtype));
}

int sap_ctrl_reset_total(int* ctrl, hipStream_t st)
{
    sap_ctrl_init_kernel<<<1, 1, 0, st>>>(ctrl, 1);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

int sap_cycles(qdw_op* op, const BlockGeom& B, int sdtype, int ncy, int nmr, void* rs,
               void* psis, void* delta, const RhsStride& bat, int nrhs, hipStream_t st, bool eo)
{
    switch (sdtype) {
    case F32: return cycles_impl<F32>(op, B, ncy, nmr, rs, psis, delta, bat, nrhs, eo, st);
    case F16S: return cycles_impl<F16S>(op, B, ncy, nmr, rs, psis, delta, bat, nrhs, eo, st);
    case BF16S: return cycles_impl<BF16S>(op, B, ncy, nmr, rs, psis, delta, bat, nrhs, eo, st);
    default: QDW_CHECK(false, QDW_EINVAL, "SAP: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    }
}

size_t sap_workspace(const qdw_op* op, int sdtype) { return 3 * spinor_bytes(op->g, sdtype) + 256; }

int sap_run(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy, int nmr,
            const BlockGeom& B, int sdtype, char* work, hipStream_t st, bool eo)
{
    switch (sdtype) {
    case F32: return sap_impl<F32>(op, rho, phi, rho_norm, ncy, nmr, B, work, eo, st);
    case F16S: return sap_impl<F16S>(op, rho, phi, rho_norm, ncy, nmr, B, work, eo, st);
    case BF16S: return sap_impl<BF16S>(op, rho, phi, rho_norm, ncy, nmr, B, work, eo, st);
    default: QDW_CHECK(false, QDW_EINVAL, "SAP: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    }
}

}  // namespace qdw

using namespace qdw;

extern "C" size_t qdw_sap_workspace_bytes(const qdw_op* op, qdw_prec sdtype)
{
    if (!op || sdtype < QDW_F32 || sdtype > QDW_BF16S) return 0;
    return sap_workspace(op, sdtype);
}

namespace {

int sap_apply_impl(const char* fn, qdw_op* op, const void* rho, void* phi, int ncy, int nmr,
                   const int bs[4], qdw_prec sdtype, void* work, size_t work_bytes,
                   void* stream, bool eo)
{
    const std::string f(fn);
    QDW_CHECK(op && rho && phi && bs && work, QDW_EINVAL, f + ": null argument");
    QDW_CHECK(rho != phi, QDW_EINVAL, f + ": rho and phi must be distinct");
    QDW_CHECK(ncy >= 0 && nmr >= 0, QDW_EINVAL, f + ": ncy and nmr must be >= 0");
    QDW_CHECK(sdtype >= QDW_F32 && sdtype <= QDW_BF16S, QDW_EINVAL,
              f + ": sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    QDW_CHECK(work_bytes >= sap_workspace(op, sdtype), QDW_EWORKSPACE,
              f + ": workspace smaller than qdw_sap_workspace_bytes()");
    BlockGeom B;
    int rc = make_block_geom(op->g, bs, &B);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_map(op, Norm2<F64>{rho, op->g.Vh}, st, op->scalars + S_TMP))) return rc;
    double n2;
    if ((rc = read_scalars(op, S_TMP, 1, &n2, st))) return rc;
    char* wk = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    return sap_run(op, rho, phi, std::sqrt(n2), ncy, nmr, B, sdtype, wk, st, eo);
}

}  // namespace

extern "C" int sap_apply(qdw_op* op, const void* rho, void* phi, int ncy, int nmr, const int bs[4],
                         qdw_prec sdtype, void* work, size_t work_bytes, void* stream)
{
    return sap_apply_impl("sap_apply", op, rho, phi, ncy, nmr, bs, sdtype, work, work_bytes,
                          stream, false);
}

extern "C" int sap_eo_apply(qdw_op* op, const void* rho, void* phi, int ncy, int nmr,
                            const int bs[4], qdw_prec sdtype, void* work, size_t work_bytes,
                            void* stream)
{
    return sap_apply_impl("sap_eo_apply", op, rho, phi, ncy, nmr, bs, sdtype, work, work_bytes,
                          stream, true);
}

extern "C" int sap_adaptive_apply(qdw_op* op, const void* rho, void* phi, int ncy_max, int nmr_max,
                                  double alpha, double tol, const int bs[4], qdw_prec sdtype,
                                  void* work, size_t work_bytes, int* cycles, int* mr_steps,
                                  void* stream)
{
    QDW_CHECK(op && rho && phi && bs && work, QDW_EINVAL, "sap_adaptive_apply: null argument");
    QDW_CHECK(rho != phi, QDW_EINVAL, "sap_adaptive_apply: rho and phi must be distinct");
    QDW_CHECK(ncy_max >= 0 && nmr_max >= 0, QDW_EINVAL,
              "sap_adaptive_apply: ncy_max and nmr_max must be >= 0");
    QDW_CHECK(alpha > 0.0 && tol >= 0.0, QDW_EINVAL, "sap_adaptive_apply: need alpha > 0, tol >= 0");
    QDW_CHECK(sdtype >= QDW_F32 && sdtype <= QDW_BF16S, QDW_EINVAL,
              "sap_adaptive_apply: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    QDW_CHECK(work_bytes >= sap_workspace(op, sdtype), QDW_EWORKSPACE,
              "sap_adaptive_apply: workspace smaller than qdw_sap_workspace_bytes()");
    BlockGeom B;
    int rc = make_block_geom(op->g, bs, &B);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_map(op, Norm2<F64>{rho, op->g.Vh}, st, op->scalars + S_TMP))) return rc;
    double n2;
    if ((rc = read_scalars(op, S_TMP, 1, &n2, st))) return rc;
    char* wk = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    int* ctrl = sap_ctrl(op, sdtype, wk);
    if ((rc = sap_ctrl_reset_total(ctrl, st))) return rc;
    if ((rc = sap_adaptive_run(op, rho, phi, std::sqrt(n2), ncy_max, nmr_max, alpha, tol, B,
                               sdtype, wk, mr_steps, st)))
        return rc;
    if (cycles) {
        QDW_HIP(hipMemcpyAsync(op->host_scalars, ctrl + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        QDW_HIP(hipStreamSynchronize(st));
        *cycles = *(const int*)op->host_scalars;
    }
    return QDW_OK;
}

// ------------------------------------------------------------------ allocation-free SAP
//
// For callers that cannot allocate device memory: the three storage-precision fields of
// the SAP application live in a file-scope device array. Its host-side name is only a
// stand-in; the device address is looked up once per device (with that device current)
// and kept.

namespace {
constexpr size_t kStaticScratchBytes = (size_t)24 << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of that device's copy

int scratch_on_current_device(char** out)
{
    int dev = -1;
    QDW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* p = nullptr;
        QDW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        QDW_CHECK(p, QDW_EDEVICE, "sap_apply_noalloc: no device address for the static scratch");
        it = g_scratch_ptr.emplace(dev, (char*)p).first;
    }
    *out = it->second;
    return QDW_OK;
}
}  // namespace

extern "C" size_t qdw_sap_noalloc_max_bytes(void) { return kStaticScratchBytes; }

extern "C" int sap_apply_noalloc(qdw_op* op, const void* rho, void* phi, int ncy, int nmr,
                                 const int bs[4], qdw_prec sdtype, void* stream)
{
    QDW_CHECK(op, QDW_EINVAL, "sap_apply_noalloc: null argument");
    QDW_CHECK(sdtype >= QDW_F32 && sdtype <= QDW_BF16S, QDW_EINVAL,
              "sap_apply_noalloc: sdtype must be QDW_F32, QDW_F16S or QDW_BF16S");
    const size_t need = sap_workspace(op, sdtype);
    QDW_CHECK(need <= kStaticScratchBytes, QDW_EWORKSPACE,
              "sap_apply_noalloc: this lattice needs " + std::to_string(need) +
                  " bytes of SAP scratch, above the static maximum of " +
                  std::to_string(kStaticScratchBytes) + " (use sap_apply with a workspace)");
    char* p = nullptr;
    if (const int rc = scratch_on_current_device(&p)) return rc;
    return sap_apply_impl("sap_apply_noalloc", op, rho, phi, ncy, nmr, bs, sdtype, p,
                          kStaticScratchBytes, stream, false);
}
