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
// components, multiplied by the link (row 2 rebuilt from rows 0, 1 and det U; the U(1)
// phase is stored inside the rows, so no trigonometry), negated when the hop crosses an
// antiperiodic time boundary, and expanded back to four spins; the factor -1/2 of the
// hopping term is applied once at the end. D^+ = gamma_5 D gamma_5 flips the projector
// signs.
//
// The eight hops form a runtime loop; for FP64 and FP32 it is software-pipelined over two
// register buffers (the loads of hop k+1 are in flight while hop k is computed). Workgroups
// walk the lattice time-slice-first within a spatial tile (walk_site). Loop-carried site indices
// pass through an empty asm statement so the optimiser cannot hoist all eight hops'
// address computations out of the loop (that would pin ~80 registers and halve the
// occupancy).
#include "qdw_host.h"
#include "dirac_core.h"

using namespace qdw;

namespace {

template <int P>
struct HopIn {
    cx<typename Traits<P>::real> s[12];  // neighbour spinor
    cx<typename Traits<P>::real> u[6];   // link rows 0, 1
    cx<typename Traits<P>::real> d;      // det of the link
};

// loads of hop k (0: +t, 1: -t, 2: +x1, ... 7: -x3) into site x = (par, i)
template <int P, int MU, bool FWD>
__device__ __forceinline__ void hop_load(const Geom& g, const void* in, const void* links,
                                         const void* dets, int par, int i, const int x[4],
                                         int lex, HopIn<P>& b)
{
    const int j = (FWD ? lex_fwd(g, x, lex, MU) : lex_bwd(g, x, lex, MU)) >> 1;
    load_spinor<P>(in, g.Vh, 1 - par, j, b.s);
    if (FWD) load_link<P>(links, dets, g.Vh, par, i, MU, b.u, b.d);       // U_mu(x)
    else load_link<P>(links, dets, g.Vh, 1 - par, j, MU, b.u, b.d);      // U_mu(x - mu)
}

// acc += U (1 -+ gamma) psi(x + mu)  or  U^+ (1 +- gamma) psi(x - mu), times the boundary
// sign (the -1/2 comes later)
template <int P, int MU, bool FWD, bool DAG>
__device__ __forceinline__ void hop_compute(const Geom& g, const int x[4], const HopIn<P>& b,
                                            cx<typename Traits<P>::real> acc[12])
{
    using R = typename Traits<P>::real;
    constexpr int SG = (FWD != DAG) ? -1 : +1;  // projector 1 + SG gamma_mu
    cx<R> h[6], w[6];
    project<R, MU, SG>(b.s, h);
    if (MU == 0 && g.bc_t < 0 && x[0] == (FWD ? g.L[0] - 1 : 0)) {
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = {-h[c].re, -h[c].im};
    }
    su3_mul<R, !FWD>(b.u, b.d, h, w);
    expand_add<R, MU, SG>(w, acc);
}

template <int P>
__device__ __forceinline__ void load_k(int k, const Geom& g, const void* in, const void* links,
                                       const void* dets, int par, int i, const int x[4], int lex,
                                       HopIn<P>& b)
{
    switch (k) {
    case 0: hop_load<P, 0, true>(g, in, links, dets, par, i, x, lex, b); break;
    case 1: hop_load<P, 0, false>(g, in, links, dets, par, i, x, lex, b); break;
    case 2: hop_load<P, 1, true>(g, in, links, dets, par, i, x, lex, b); break;
    case 3: hop_load<P, 1, false>(g, in, links, dets, par, i, x, lex, b); break;
    case 4: hop_load<P, 2, true>(g, in, links, dets, par, i, x, lex, b); break;
    case 5: hop_load<P, 2, false>(g, in, links, dets, par, i, x, lex, b); break;
    case 6: hop_load<P, 3, true>(g, in, links, dets, par, i, x, lex, b); break;
    default: hop_load<P, 3, false>(g, in, links, dets, par, i, x, lex, b); break;
    }
}

template <int P, bool DAG>
__device__ __forceinline__ void compute_k(int k, const Geom& g, const int x[4], const HopIn<P>& b,
                                          cx<typename Traits<P>::real> acc[12])
{
    switch (k) {
    case 0: hop_compute<P, 0, true, DAG>(g, x, b, acc); break;
    case 1: hop_compute<P, 0, false, DAG>(g, x, b, acc); break;
    case 2: hop_compute<P, 1, true, DAG>(g, x, b, acc); break;
    case 3: hop_compute<P, 1, false, DAG>(g, x, b, acc); break;
    case 4: hop_compute<P, 2, true, DAG>(g, x, b, acc); break;
    case 5: hop_compute<P, 2, false, DAG>(g, x, b, acc); break;
    case 6: hop_compute<P, 3, true, DAG>(g, x, b, acc); break;
    default: hop_compute<P, 3, false, DAG>(g, x, b, acc); break;
    }
}

template <int P, bool DAG>
__global__ __launch_bounds__(256) void dw_kernel(Geom g, const void* __restrict__ in,
                                                 void* __restrict__ out,
                                                 const void* __restrict__ links,
                                                 const void* __restrict__ dets,
                                                 const void* __restrict__ clover)
{
    using R = typename Traits<P>::real;
    const int par = threadIdx.x >> 7;
    int i;
    if (!walk_site(g, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x & 127, i)) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<R> hop[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hop[c] = {(R)0, (R)0};
    if constexpr (P == F64 || P == F32) {
        // bandwidth-bound formats: two buffers, loads of the next hop in flight
        HopIn<P> A, B;
        load_k<P>(0, g, in, links, dets, par, i, x, lex, A);
#pragma unroll 1
        for (int k = 0; k < 8; k += 2) {
            int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
            load_k<P>(k + 1, g, in, links, dets, par, ii, xx, ll, B);
            compute_k<P, DAG>(k, g, xx, A, hop);
            if (k + 2 < 8) load_k<P>(k + 2, g, in, links, dets, par, ii, xx, ll, A);
            compute_k<P, DAG>(k + 1, g, xx, B, hop);
        }
    } else {
        // 16-bit storage is limited by the conversions and arithmetic, not by loads: one
        // buffer keeps the register count (and so the occupancy) lower
        HopIn<P> A;
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
            load_k<P>(k, g, in, links, dets, par, ii, xx, ll, A);
            compute_k<P, DAG>(k, g, xx, A, hop);
        }
    }
    cx<R> s[12], acc[12];
    load_spinor<P>(in, g.Vh, par, i, s);
    clover_apply<P>(clover, g.Vh, par, i, s, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = acc[c] - scale(hop[c], (R)0.5);
    store_spinor<P>(out, g.Vh, par, i, acc);
}

template <int P, bool DAG>
int launch(qdw_op* op, const void* in, void* out, hipStream_t st)
{
    const Geom& g = op->g;
    dw_kernel<P, DAG><<<walk_blocks(g), 256, 0, st>>>(g, in, out, op->links[P], op->det[P],
                                                      op->clover[P]);
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
