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
#include "dirac_core.h"

using namespace qdw;

namespace {

// one hop into site x = (par, i): FWD: U_mu(x) (1 -+ gamma) psi(x + mu), link owned by x;
// backward: U_mu(x - mu)^+ (1 +- gamma) psi(x - mu), link owned by x - mu
template <int P, int MU, bool FWD, bool DAG>
__device__ __forceinline__ void hop(const Geom& g, const void* in, const void* links,
                                    const void* theta, int par, int i, const int x[4], int lex,
                                    cx<typename Traits<P>::real> acc[12])
{
    using R = typename Traits<P>::real;
    constexpr int SG = (FWD != DAG) ? -1 : +1;  // projector 1 + SG gamma_mu
    cx<R> s[12], h[6], w[6], u[6], ph;
    const int j = (FWD ? lex_fwd(g, x, lex, MU) : lex_bwd(g, x, lex, MU)) >> 1;
    load_spinor<P>(in, g.Vh, 1 - par, j, s);
    project<R, MU, SG>(s, h);
    if (FWD) {
        load_link<P>(links, theta, g.Vh, par, i, MU, u, ph);
        const R sg = (MU == 0 && x[0] == g.L[0] - 1) ? (R)(-0.5 * g.bc_t) : (R)-0.5;
        su3_apply<R, false>(u, scale(ph, sg), h, w);
    } else {
        load_link<P>(links, theta, g.Vh, 1 - par, j, MU, u, ph);
        const R sg = (MU == 0 && x[0] == 0) ? (R)(-0.5 * g.bc_t) : (R)-0.5;
        su3_apply<R, true>(u, scale(conj_(ph), sg), h, w);
    }
    expand_add<R, MU, SG>(w, acc);
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
    // the eight hops one at a time (a runtime loop keeps the compiler from hoisting all
    // eight neighbour loads at once, which would exhaust the register file)
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        switch (k) {
        case 0: hop<P, 0, true, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 1: hop<P, 0, false, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 2: hop<P, 1, true, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 3: hop<P, 1, false, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 4: hop<P, 2, true, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 5: hop<P, 2, false, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        case 6: hop<P, 3, true, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        default: hop<P, 3, false, DAG>(g, in, links, theta, par, i, x, lex, acc); break;
        }
    }
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
