// dirac.hip -- the Wilson-clover operator D and D^+ on eo-SoA fields.
//
// One lane per output site; a workgroup of 2*ts lanes owns ts consecutive even-odd
// indices of one time slice in BOTH parities (lanes 0..ts-1 even, ts..2ts-1 odd). The even
// site with index i and the odd site with index i are lexicographic neighbours along x3,
// so a workgroup covers a compact run of the lattice: the eight links a site reads are
// mostly the same links its neighbours in the workgroup read (every link joins an even and
// an odd site), and the neighbour spinors are shared through L1/L2. Workgroups are mapped
// XCD-contiguously and walk time-slice-first within a spatial tile (walk_site).
//
// Per hop the neighbour spinor is spin-projected with (1 -+ gamma_mu) to two spin
// components, multiplied by the link (row 2 rebuilt from rows 0, 1 and det U; the U(1)
// phase is stored inside the rows, so no trigonometry), negated when the hop crosses an
// antiperiodic time boundary, and expanded back to four spins; the factor -1/2 of the
// hopping term is applied once at the end. D^+ = gamma_5 D gamma_5 flips the projector
// signs.
//
// The eight hops form a runtime loop; optionally (PIPE) it is software-pipelined over two
// register buffers: the loads of hop k+1 are in flight while hop k is computed. Loop-carried
// site indices pass through an empty asm statement so the optimiser cannot hoist all eight
// hops' address computations out of the loop (that would pin ~80 registers and halve the
// occupancy).
//
// Several right-hand sides on one operator (a table of up to kMaxRhs fields) run in one
// launch with the right-hand side as the fastest-varying workgroup index: the workgroups
// that read a tile's links and clover blocks for different right-hand sides run together,
// so L2 serves those bytes once for all of them.
#include <chrono>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "qdw_host.h"
#include "dirac_core.h"

using namespace qdw;

namespace qdw {
struct RhsTable {
    const void* in[kMaxRhs];
    void* out[kMaxRhs];
    const int* gate;  // optional: right-hand side r is skipped when gate[r * gstride] == 0
    int gstride;
};
}  // namespace qdw

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
// sign; with HALF the term is scaled by -1/2 (the hopping term's factor) before it is added
template <int P, int MU, bool FWD, bool DAG, bool HALF = false>
__device__ __forceinline__ void hop_compute(const Geom& g, const int x[4], const HopIn<P>& b,
                                            cx<typename Traits<P>::real> acc[12])
{
    using R = typename Traits<P>::real;
    constexpr int SG = (FWD != DAG) ? -1 : +1;  // projector 1 + SG gamma_mu
    cx<R> h[6], w[6];
    project<R, MU, SG>(b.s, h);
    const bool flip = MU == 0 && g.bc_t < 0 && x[0] == (FWD ? g.L[0] - 1 : 0);
    if (HALF) {
        const R f = flip ? (R)0.5 : (R)-0.5;
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = scale(h[c], f);
    } else if (flip) {
#pragma unroll
        for (int c = 0; c < 6; ++c) h[c] = -h[c];
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

template <int P, bool DAG, bool HALF = false>
__device__ __forceinline__ void compute_k(int k, const Geom& g, const int x[4], const HopIn<P>& b,
                                          cx<typename Traits<P>::real> acc[12])
{
    switch (k) {
    case 0: hop_compute<P, 0, true, DAG, HALF>(g, x, b, acc); break;
    case 1: hop_compute<P, 0, false, DAG, HALF>(g, x, b, acc); break;
    case 2: hop_compute<P, 1, true, DAG, HALF>(g, x, b, acc); break;
    case 3: hop_compute<P, 1, false, DAG, HALF>(g, x, b, acc); break;
    case 4: hop_compute<P, 2, true, DAG, HALF>(g, x, b, acc); break;
    case 5: hop_compute<P, 2, false, DAG, HALF>(g, x, b, acc); break;
    case 6: hop_compute<P, 3, true, DAG, HALF>(g, x, b, acc); break;
    default: hop_compute<P, 3, false, DAG, HALF>(g, x, b, acc); break;
    }
}

// One lane per site. With half-precision storage and no software pipelining the kernel
// fits four waves per SIMD without spilling (123 VGPRs instead of 156 at three), which
// hides more of the gather latency.
template <int P, bool DAG, bool PIPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P >= F16S && !PIPE ? 4 : 1)))
void dw_kernel(Geom g, RhsTable tab, int nrhs, const void* __restrict__ links,
               const void* __restrict__ dets, const void* __restrict__ clover)
{
    using R = typename Traits<P>::real;
    const int logical = xcd_tile(blockIdx.x, gridDim.x);
    const int tile = logical / nrhs;
    const int rhs = logical - tile * nrhs;
    if (tab.gate && !tab.gate[(long)rhs * tab.gstride]) return;
    const void* __restrict__ in = tab.in[rhs];
    void* __restrict__ out = tab.out[rhs];
    int par, i;
    if (!walk_site(g, tile, threadIdx.x, par, i)) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<R> hop[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hop[c] = {(R)0, (R)0};
    if constexpr (PIPE) {
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
    clover54_apply<P>(clover, g.Vh, par, i, (R)g.cdiag, s, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = acc[c] - scale(hop[c], (R)0.5);
    store_spinor<P>(out, g.Vh, par, i, acc);
}

// Marching form: a workgroup owns one spatial tile (both parities) and walks the nt time
// slices of its chunk in order. The time hops then never go to memory twice:
//   * +t: at step t every lane loads the spinor its own lane will need at t+1; projected
//     with the +t projector it is exactly the +t neighbour of the partner lane (the other
//     parity, same even-odd index: the same spatial point one slice down), so it goes to
//     the partner through LDS;
//   * -t: at the end of step t each lane has its own spinor and its own forward t link in
//     hand; it forms U_0^+ (1 -+ gamma_0) psi, the -t hop of the partner's site at t+1,
//     and hands it over through LDS.
// The lane's own spinor of a slice is loaded once, as the +t neighbour one step earlier,
// and kept in registers for the clover term and the hand-over (a reload a step later
// would find it evicted from L2); the t link likewise within a step.
// Only the spatial hops read neighbours from memory, and they are done one step early: in
// the step that loads slice t+1 (every lane its own site, all workgroups of an XCD at about
// the same time), the lane also forms A psi and the six spatial hops of its site at t+1,
// while those spinors are still in L2; the time hops are added in the next step, once the
// partner has handed them over. Gathering a slice in the step after it was loaded found
// most of it evicted (an XCD streams more than its 4 MB L2 per step) and read it from HBM
// a second time. One barrier per step: the LDS buffers are double-buffered by slice
// parity (see the step comments).
template <int P, bool DAG, bool PIPE>
__device__ __forceinline__ void march_site_hops(const Geom& g, const void* in, const void* links,
                                                const void* dets, int par, int i, const int x[4],
                                                int lex, cx<typename Traits<P>::real> acc[12])
{
    if constexpr (!PIPE) {
        // the six spatial hops (loop steps 2..7 of dw_kernel), one register buffer
        HopIn<P> A;
#pragma unroll 1
        for (int k = 2; k < 8; ++k) {
            int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
            load_k<P>(k, g, in, links, dets, par, ii, xx, ll, A);
            compute_k<P, DAG, true>(k, g, xx, A, acc);
        }
        return;
    }
    // the six spatial hops (loop steps 2..7 of dw_kernel), two register buffers
    HopIn<P> A, B;
    load_k<P>(2, g, in, links, dets, par, i, x, lex, A);
#pragma unroll 1
    for (int k = 2; k < 8; k += 2) {
        int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
        asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
        load_k<P>(k + 1, g, in, links, dets, par, ii, xx, ll, B);
        compute_k<P, DAG, true>(k, g, xx, A, acc);
        if (k + 2 < 8) load_k<P>(k + 2, g, in, links, dets, par, ii, xx, ll, A);
        compute_k<P, DAG, true>(k + 1, g, xx, B, acc);
    }
}

template <int P, bool DAG, bool PIPE>
__global__ __launch_bounds__(256) void dw_march_kernel(Geom g, RhsTable tab, int nrhs,
                                                       const void* __restrict__ links,
                                                       const void* __restrict__ dets,
                                                       const void* __restrict__ clover)
{
    using R = typename Traits<P>::real;
    constexpr int SGF = DAG ? +1 : -1;  // projector of the +t hop: 1 + SGF gamma_0
    constexpr int SGB = -SGF;           // of the -t hop
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int nl = blockDim.x;  // 2 ts lanes
    R* hp = (R*)smem;           // [2 slots][12 reals][nl]: projected +t neighbours
    R* pw = hp + 2 * 12 * nl;   // [2 slots][12 reals][nl]: transported -t neighbours
    const int logical = xcd_tile(blockIdx.x, gridDim.x);
    const int wg = logical / nrhs;
    const int rhs = logical - wg * nrhs;
    if (tab.gate && !tab.gate[(long)rhs * tab.gstride]) return;  // the whole workgroup
    const void* __restrict__ in = tab.in[rhs];
    void* __restrict__ out = tab.out[rhs];
    const int c = wg / g.ntile, s = wg - c * g.ntile;
    const int t0 = c * g.nt;
    const int tid = threadIdx.x;
    const int par = tid >= g.ts ? 1 : 0;
    const int lane = tid - par * g.ts;
    const int partner = tid + (par ? -g.ts : g.ts);
    int k;
    bool valid;
    if (g.walk == 0) {
        k = s * g.ts + lane;
        valid = k < g.S;
    } else {
        const int b = s / g.L[1], x1 = s - b * g.L[1];
        k = x1 * g.slab + b * g.ts + lane;
        valid = b * g.ts + lane < g.slab;
    }
    auto put6 = [&](R* buf, int slot, int who, const cx<R> v[6]) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            buf[(slot * 12 + 2 * q) * nl + who] = v[q].re;
            buf[(slot * 12 + 2 * q + 1) * nl + who] = v[q].im;
        }
    };
    auto get6 = [&](const R* buf, int slot, cx<R> v[6]) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            v[q] = {buf[(slot * 12 + 2 * q) * nl + tid], buf[(slot * 12 + 2 * q + 1) * nl + tid]};
    };
    // U_0(y)^+ (1 + SGB gamma_0) psi(y) for the partner's site one slice up (sign when the
    // hop wraps from T-1 to 0)
    auto push = [&](int t, int slot, const cx<R> sp[12], const cx<R> u[6], cx<R> d) {
        cx<R> h[6], w[6];
        project<R, 0, SGB>(sp, h);
        if (g.bc_t < 0 && t == g.L[0] - 1) {
#pragma unroll
            for (int q = 0; q < 6; ++q) h[q] = {-h[q].re, -h[q].im};
        }
        su3_mul<R, true>(u, d, h, w);
        put6(pw, slot, partner, w);
    };
    // A psi plus the six spatial hops (scaled by -1/2) of this lane's site at slice tt,
    // whose spinor `sp` the lane holds
    auto site_part = [&](int tt, const cx<R> sp[12], cx<R> acc[12]) {
        const int i = tt * g.S + k;
        int x[4], lex;
        eo_coords(g, par, i, x, lex);
        clover54_apply<P>(clover, g.Vh, par, i, (R)g.cdiag, sp, acc);
        march_site_hops<P, DAG, PIPE>(g, in, links, dets, par, i, x, lex, acc);
    };
    // the lane's own spinor of the current slice stays in registers from the step that
    // loaded it for the partner (a reload one step later would come from HBM again), and
    // so does the accumulator of the current slice, begun in the step before
    cx<R> own[12], acc[12];
    if (valid) {
        const int tp = t0 == 0 ? g.L[0] - 1 : t0 - 1;
        cx<R> u[6], d;
        load_spinor<P>(in, g.Vh, par, tp * g.S + k, own);
        load_link<P>(links, dets, g.Vh, par, tp * g.S + k, 0, u, d);
        push(tp, t0 & 1, own, u, d);
        load_spinor<P>(in, g.Vh, par, t0 * g.S + k, own);
        site_part(t0, own, acc);
    }
    for (int step = 0; step < g.nt; ++step) {
        const int t = t0 + step;
        const int tn = t + 1 == g.L[0] ? 0 : t + 1;
        // (1) the spinor this lane owns at t+1, projected for the partner's +t hop; slot
        //     (t+1)&1 was last read two steps ago, before the previous barrier
        cx<R> nxt[12];
        if (valid) {
            cx<R> h[6];
            load_spinor<P>(in, g.Vh, par, tn * g.S + k, nxt);
            project<R, 0, SGF>(nxt, h);
            put6(hp, (t + 1) & 1, partner, h);
        }
        __syncthreads();
        if (valid) {
            const int i = t * g.S + k;
            const int x0 = t;  // the time coordinate of the site
            // the site's forward t link serves the +t hop and the hand-over below
            cx<R> u0[6], d0;
            load_link<P>(links, dets, g.Vh, par, i, 0, u0, d0);
            // (2) the partner's -t hop at t+1; slot (t+1)&1 was read one step ago, before
            //     this step's barrier
            if (step + 1 < g.nt) push(t, (t + 1) & 1, own, u0, d0);
            {
                // +t: U_0(x) times the projected neighbour from the partner
                cx<R> h[6], w[6];
                get6(hp, (t + 1) & 1, h);
                const R f = (g.bc_t < 0 && x0 == g.L[0] - 1) ? (R)0.5 : (R)-0.5;
#pragma unroll
                for (int q = 0; q < 6; ++q) h[q] = scale(h[q], f);
                su3_mul<R, false>(u0, d0, h, w);
                expand_add<R, 0, SGF>(w, acc);
                // -t: already transported by the partner
                get6(pw, t & 1, w);
#pragma unroll
                for (int q = 0; q < 6; ++q) w[q] = scale(w[q], (R)-0.5);
                expand_add<R, 0, SGB>(w, acc);
            }
            store_spinor<P>(out, g.Vh, par, i, acc);
            // (3) the next slice's clover term and spatial hops, on the spinors loaded in
            //     this step
            if (step + 1 < g.nt) {
#pragma unroll
                for (int q = 0; q < 12; ++q) own[q] = nxt[q];
                site_part(tn, own, acc);
            }
        }
    }
}

// Even-odd reduced operator D^ = A_ee - D_eo A_oo^-1 D_oe on the even half of a field, in
// two passes over one parity each (one lane per site):
//   stage 1, odd sites:  t = A_oo^-1 (D_oe psi_e) = A_oo^-1 (-1/2 sum of the hops of psi_e)
//   stage 2, even sites: out = A_ee psi_e - D_eo t = A_ee psi_e + 1/2 sum of the hops of t
// t lives in the odd half of the output field. D^+ = gamma_5 D^ gamma_5 flips the
// projector signs as for D (A and A^-1 commute with gamma_5).
template <int P, bool DAG, int STAGE, bool PIPE>
__global__ __launch_bounds__(256) void schur_kernel(Geom g, int ntile1, const void* hsrc,
                                                    const void* dsrc, void* out,
                                                    const void* __restrict__ links,
                                                    const void* __restrict__ dets,
                                                    const void* __restrict__ diag)
{
    using R = typename Traits<P>::real;
    constexpr int par = STAGE == 1 ? 1 : 0;
    // one parity: tiles of 256 consecutive even-odd indices of a slice, nt slices of one
    // tile in a row, XCD-contiguous (as the one-workgroup-per-slice D kernel, walk 0)
    const int logical = xcd_tile(blockIdx.x, gridDim.x);
    const int per_chunk = g.nt * ntile1;
    const int c = logical / per_chunk;
    const int r = logical - c * per_chunk;
    const int sidx = r / g.nt;
    const int t = c * g.nt + (r - sidx * g.nt);
    const int k = sidx * 256 + (int)threadIdx.x;
    if (k >= g.S) return;
    const int i = t * g.S + k;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<R> hop[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) hop[q] = {(R)0, (R)0};
    if constexpr (PIPE) {
        HopIn<P> A, B;
        load_k<P>(0, g, hsrc, links, dets, par, i, x, lex, A);
#pragma unroll 1
        for (int kk = 0; kk < 8; kk += 2) {
            int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
            load_k<P>(kk + 1, g, hsrc, links, dets, par, ii, xx, ll, B);
            compute_k<P, DAG>(kk, g, xx, A, hop);
            if (kk + 2 < 8) load_k<P>(kk + 2, g, hsrc, links, dets, par, ii, xx, ll, A);
            compute_k<P, DAG>(kk + 1, g, xx, B, hop);
        }
    } else {
        HopIn<P> A;
#pragma unroll 1
        for (int kk = 0; kk < 8; ++kk) {
            int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
            asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
            load_k<P>(kk, g, hsrc, links, dets, par, ii, xx, ll, A);
            compute_k<P, DAG>(kk, g, xx, A, hop);
        }
    }
    cx<R> acc[12];
    if constexpr (STAGE == 1) {
#pragma unroll
        for (int q = 0; q < 12; ++q) hop[q] = scale(hop[q], (R)-0.5);
        clover_apply<P>(diag, g.Vh, par, i, hop, acc);
    } else {
        cx<R> sp[12];
        load_spinor<P>(dsrc, g.Vh, par, i, sp);
        clover_apply<P>(diag, g.Vh, par, i, sp, acc);
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[q] = acc[q] + scale(hop[q], (R)0.5);
    }
    store_spinor<P>(out, g.Vh, par, i, acc);
}

template <int P, bool DAG>
int schur_launch_t(qdw_op* op, const void* in, void* out, hipStream_t st)
{
    const Geom& g = op->g;
    const int ntile1 = (g.S + 255) / 256;
    const int nb = g.L[0] * ntile1;
    // the hop loop is software-pipelined where the registers allow it (FP64, FP32), as for D
    constexpr bool PIPE = P == F64 || P == F32;
    schur_kernel<P, DAG, 1, PIPE><<<nb, 256, 0, st>>>(g, ntile1, in, nullptr, out, op->links[P],
                                                      op->det[P], op->cloverinv[P]);
    QDW_LAUNCH_CHECK();
    schur_kernel<P, DAG, 2, PIPE><<<nb, 256, 0, st>>>(g, ntile1, out, in, out, op->links[P],
                                                      op->det[P], op->clover[P]);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

// the operator's geometry with the D kernel's own shape for precision P
inline Geom shaped(const qdw_op* op, int P)
{
    Geom g = op->g;
    set_walk(g, op->dw_shape[P].ts, op->dw_shape[P].nt, op->dw_shape[P].walk);
    return g;
}

template <int P, bool DAG>
int launch(qdw_op* op, const RhsTable& tab, int nrhs, hipStream_t st)
{
    const Geom g = shaped(op, P);
    if (op->dw_shape[P].march) {
        using R = typename Traits<P>::real;
        const int nblk = (g.L[0] / g.nt) * g.ntile * nrhs;
        const size_t lds = (size_t)2 * 2 * 12 * (2 * g.ts) * sizeof(R);
        static_assert(sizeof(R) == 8 || sizeof(R) == 4, "real type");
        if (op->dw_shape[P].pipe)
            dw_march_kernel<P, DAG, true><<<nblk, 2 * g.ts, lds, st>>>(g, tab, nrhs, op->links[P],
                                                                       op->det[P], op->clover54[P]);
        else
            dw_march_kernel<P, DAG, false><<<nblk, 2 * g.ts, lds, st>>>(g, tab, nrhs, op->links[P],
                                                                        op->det[P], op->clover54[P]);
        QDW_LAUNCH_CHECK();
        return QDW_OK;
    }
    const int nblk = walk_blocks(g) * nrhs;
    if (op->dw_shape[P].pipe)
        dw_kernel<P, DAG, true><<<nblk, 2 * g.ts, 0, st>>>(g, tab, nrhs, op->links[P], op->det[P],
                                                           op->clover54[P]);
    else
        dw_kernel<P, DAG, false><<<nblk, 2 * g.ts, 0, st>>>(g, tab, nrhs, op->links[P], op->det[P],
                                                            op->clover54[P]);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

int dispatch(qdw_op* op, const RhsTable& tab, int nrhs, int prec, bool dag, hipStream_t st)
{
    switch (prec) {
    case QDW_F64: return dag ? launch<F64, true>(op, tab, nrhs, st) : launch<F64, false>(op, tab, nrhs, st);
    case QDW_F32: return dag ? launch<F32, true>(op, tab, nrhs, st) : launch<F32, false>(op, tab, nrhs, st);
    case QDW_F16S: return dag ? launch<F16S, true>(op, tab, nrhs, st) : launch<F16S, false>(op, tab, nrhs, st);
    case QDW_BF16S: return dag ? launch<BF16S, true>(op, tab, nrhs, st) : launch<BF16S, false>(op, tab, nrhs, st);
    default: QDW_CHECK(false, QDW_EINVAL, "dw_apply: bad precision");
    }
}

// ------------------------------------------------------------------ uncompressed control
//
// The same operator with every FP64 link read as its full 3x3 matrix (18 reals, 9 chunks
// per link, no row rebuilt in the kernel): the control for the two-row storage. Only the
// one-lane-per-site form with a plain hop loop exists for it; it takes the walk of the
// operator's FP64 shape when that is a one-lane-per-site shape, else 128-site tiles in
// chunks of 4 slices, and is compared with the compressed kernel in the same form.

// full links, [par * 4 + mu][site / 64][9][site % 64] chunks of one complex number each:
// rows 0, 1 as stored and row 2 = d conj(row0 x row1), formed as the compressed kernels
// form it
__global__ __launch_bounds__(256) void full_links_kernel(Geom g, const void* links, const void* dets,
                                                         void* full)
{
    const long n = (long)g.Vh * 8;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int row = (int)(q / g.Vh), i = (int)(q - (long)row * g.Vh);
        cx<double> u[6], d;
        load_link<F64>(links, dets, g.Vh, row >> 2, i, row & 3, u, d);
        const cx<double> m[9] = {u[0], u[1], u[2], u[3], u[4], u[5],
                                 d * conj_(cmadd(u[1] * u[5], -u[2], u[4])),
                                 d * conj_(cmadd(u[2] * u[3], -u[0], u[5])),
                                 d * conj_(cmadd(u[0] * u[4], -u[1], u[3]))};
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            Chunk<F64> c;
            c.v[0] = m[k].re;
            c.v[1] = m[k].im;
            store_chunk<F64>(full, chunk_at(g.Vh, 9, row, k, i), c);
        }
    }
}

template <bool DAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
void dw_full_kernel(Geom g, const void* __restrict__ in, void* __restrict__ out,
                    const void* __restrict__ full, const void* __restrict__ clover)
{
    int par, i;
    if (!walk_site(g, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, par, i)) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<double> hop[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hop[c] = {0.0, 0.0};
    auto one = [&](auto mu_c, auto fwd_c, int ii, int ll, const int xx[4]) {
        constexpr int MU = decltype(mu_c)::value;
        constexpr bool FWD = decltype(fwd_c)::value;
        constexpr int SG = (FWD != DAG) ? -1 : +1;
        const int j = (FWD ? lex_fwd(g, xx, ll, MU) : lex_bwd(g, xx, ll, MU)) >> 1;
        cx<double> sp[12], m[9], h[6], w[6];
        load_spinor<F64>(in, g.Vh, 1 - par, j, sp);
        const int lrow = (FWD ? par : 1 - par) * 4 + MU, li = FWD ? ii : j;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const Chunk<F64> c = load_chunk_cached<F64>(full, chunk_at(g.Vh, 9, lrow, k, li));
            m[k] = {c.v[0], c.v[1]};
        }
        project<double, MU, SG>(sp, h);
        if (MU == 0 && g.bc_t < 0 && xx[0] == (FWD ? g.L[0] - 1 : 0)) {
#pragma unroll
            for (int c = 0; c < 6; ++c) h[c] = -h[c];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const cx<double> h0 = h[3 * a], h1 = h[3 * a + 1], h2 = h[3 * a + 2];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                if (FWD)
                    w[3 * a + r] = cmadd(cmadd(m[3 * r] * h0, m[3 * r + 1], h1), m[3 * r + 2], h2);
                else
                    w[3 * a + r] = cmadd_conj(cmadd_conj(cmul_conj(m[r], h0), m[3 + r], h1), m[6 + r], h2);
            }
        }
        expand_add<double, MU, SG>(w, hop);
    };
    // the eight hops as a runtime loop over opaque site indices (as dw_kernel)
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        int ii = i, ll = lex, xx[4] = {x[0], x[1], x[2], x[3]};
        asm volatile("" : "+v"(ii), "+v"(ll), "+v"(xx[0]), "+v"(xx[1]), "+v"(xx[2]), "+v"(xx[3]));
        using T = std::true_type;
        using F = std::false_type;
        switch (k) {
        case 0: one(std::integral_constant<int, 0>{}, T{}, ii, ll, xx); break;
        case 1: one(std::integral_constant<int, 0>{}, F{}, ii, ll, xx); break;
        case 2: one(std::integral_constant<int, 1>{}, T{}, ii, ll, xx); break;
        case 3: one(std::integral_constant<int, 1>{}, F{}, ii, ll, xx); break;
        case 4: one(std::integral_constant<int, 2>{}, T{}, ii, ll, xx); break;
        case 5: one(std::integral_constant<int, 2>{}, F{}, ii, ll, xx); break;
        case 6: one(std::integral_constant<int, 3>{}, T{}, ii, ll, xx); break;
        default: one(std::integral_constant<int, 3>{}, F{}, ii, ll, xx); break;
        }
    }
    cx<double> sp[12], acc[12];
    load_spinor<F64>(in, g.Vh, par, i, sp);
    clover54_apply<F64>(clover, g.Vh, par, i, g.cdiag, sp, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = acc[c] - scale(hop[c], 0.5);
    store_spinor<F64>(out, g.Vh, par, i, acc);
}

int apply_checked(qdw_op* op, const void* in, void* out, qdw_prec prec, bool dag, void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_apply: null argument");
    QDW_CHECK(in != out, QDW_EINVAL, "dw_apply: in and out must be distinct fields");
    RhsTable tab{};
    tab.in[0] = in;
    tab.out[0] = out;
    return dispatch(op, tab, 1, prec, dag, (hipStream_t)stream);
}

}  // namespace

namespace qdw {
// internal entries used by the solvers (same kernels, no argument re-validation)
int dw_launch(qdw_op* op, const void* in, void* out, int prec, bool dag, hipStream_t st)
{
    RhsTable tab{};
    tab.in[0] = in;
    tab.out[0] = out;
    return dispatch(op, tab, 1, prec, dag, st);
}

int schur_launch(qdw_op* op, const void* in, void* out, int prec, bool dag, hipStream_t st)
{
    switch (prec) {
    case F64: return dag ? schur_launch_t<F64, true>(op, in, out, st) : schur_launch_t<F64, false>(op, in, out, st);
    case F32: return dag ? schur_launch_t<F32, true>(op, in, out, st) : schur_launch_t<F32, false>(op, in, out, st);
    case F16S: return dag ? schur_launch_t<F16S, true>(op, in, out, st) : schur_launch_t<F16S, false>(op, in, out, st);
    case BF16S: return dag ? schur_launch_t<BF16S, true>(op, in, out, st) : schur_launch_t<BF16S, false>(op, in, out, st);
    default: QDW_CHECK(false, QDW_EINVAL, "schur: bad precision");
    }
}

int dw_launch_multi(qdw_op* op, const void* const* in, void* const* out, int nrhs, int prec,
                    bool dag, const int* gate, int gstride, hipStream_t st)
{
    RhsTable tab{};
    tab.gate = gate;
    tab.gstride = gstride;
    for (int r = 0; r < nrhs; ++r) {
        tab.in[r] = in[r];
        tab.out[r] = out[r];
    }
    return dispatch(op, tab, nrhs, prec, dag, st);
}
}  // namespace qdw

extern "C" int dw_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    return apply_checked(op, in, out, prec, false, stream);
}

extern "C" int dw_dag_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    return apply_checked(op, in, out, prec, true, stream);
}

extern "C" size_t qdw_full_links_bytes(const qdw_op* op)
{
    return op ? (size_t)padded(op->g.Vh) * 8 * 9 * 16 : 0;
}

extern "C" int qdw_set_full_links(qdw_op* op, void* dev_mem, size_t bytes, void* stream)
{
    QDW_CHECK(op && dev_mem, QDW_EINVAL, "qdw_set_full_links: null argument");
    QDW_CHECK(bytes >= qdw_full_links_bytes(op), QDW_EWORKSPACE,
              "qdw_set_full_links: block smaller than qdw_full_links_bytes()");
    QDW_CHECK(((uintptr_t)dev_mem & 15) == 0, QDW_EINVAL,
              "qdw_set_full_links: the block must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    full_links_kernel<<<1024, 256, 0, st>>>(op->g, op->links[F64], op->det[F64], dev_mem);
    QDW_LAUNCH_CHECK();
    op->full_links = dev_mem;
    return QDW_OK;
}

extern "C" int dw_apply_full_links(qdw_op* op, const void* in, void* out, int dagger, void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_apply_full_links: null argument");
    QDW_CHECK(in != out, QDW_EINVAL, "dw_apply_full_links: in and out must be distinct fields");
    QDW_CHECK(op->full_links, QDW_EINVAL,
              "dw_apply_full_links: no full links (call qdw_set_full_links first)");
    Geom g = op->g;
    const auto& sh = op->dw_shape[F64];
    if (sh.march) set_walk(g, 128, g.L[0] % 4 == 0 ? 4 : 1, 0);
    else set_walk(g, sh.ts, sh.nt, sh.walk);
    hipStream_t st = (hipStream_t)stream;
    if (dagger)
        dw_full_kernel<true><<<walk_blocks(g), 2 * g.ts, 0, st>>>(g, in, out, op->full_links,
                                                                   op->clover54[F64]);
    else
        dw_full_kernel<false><<<walk_blocks(g), 2 * g.ts, 0, st>>>(g, in, out, op->full_links,
                                                                    op->clover54[F64]);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

extern "C" int dw_schur_apply(qdw_op* op, const void* in, void* out, qdw_prec prec, void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_schur_apply: null argument");
    QDW_CHECK(in != out, QDW_EINVAL, "dw_schur_apply: in and out must be distinct fields");
    return qdw::schur_launch(op, in, out, prec, false, (hipStream_t)stream);
}

extern "C" int dw_schur_dag_apply(qdw_op* op, const void* in, void* out, qdw_prec prec,
                                  void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_schur_dag_apply: null argument");
    QDW_CHECK(in != out, QDW_EINVAL, "dw_schur_dag_apply: in and out must be distinct fields");
    return qdw::schur_launch(op, in, out, prec, true, (hipStream_t)stream);
}

extern "C" int dw_apply_multi(qdw_op* op, const void* const* in, void* const* out, int nrhs,
                              qdw_prec prec, void* stream)
{
    QDW_CHECK(op && in && out, QDW_EINVAL, "dw_apply_multi: null argument");
    QDW_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, QDW_EINVAL, "dw_apply_multi: need 1 <= nrhs <= 64");
    for (int r = 0; r < nrhs; ++r) {
        QDW_CHECK(in[r] && out[r], QDW_EINVAL, "dw_apply_multi: null field");
        for (int q = 0; q < nrhs; ++q)
            QDW_CHECK(in[r] != out[q], QDW_EINVAL, "dw_apply_multi: an output aliases an input");
    }
    return qdw::dw_launch_multi(op, in, out, nrhs, prec, false, nullptr, 0, (hipStream_t)stream);
}

// ------------------------------------------------------------------ shapes and autotuner

namespace {
// timing input of the autotuner: every stored value a hashed number in [-0.5, 0.5) (all-zero
// fields would time a faster memory path than real data)
template <int P>
__global__ void fill_pattern_kernel(void* buf, long n)
{
    using S = typename Traits<P>::store;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)j * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        const float v = (float)(h & 0xFFFFu) * (1.0f / 65536.0f) - 0.5f;
        ((S*)buf)[j] = to_store<P>((typename Traits<P>::real)v);
    }
}

int fill_pattern(void* buf, size_t bytes, int prec, hipStream_t st)
{
    switch (prec) {
    case F64: fill_pattern_kernel<F64><<<1024, 256, 0, st>>>(buf, (long)(bytes / 8)); break;
    case F32: fill_pattern_kernel<F32><<<1024, 256, 0, st>>>(buf, (long)(bytes / 4)); break;
    case F16S: fill_pattern_kernel<F16S><<<1024, 256, 0, st>>>(buf, (long)(bytes / 2)); break;
    default: fill_pattern_kernel<BF16S><<<1024, 256, 0, st>>>(buf, (long)(bytes / 2)); break;
    }
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

// LDS of a marching workgroup: two double-buffered hand-over arrays of 12 reals per lane
inline size_t march_lds(int prec, int ts) { return (size_t)96 * ts * (prec == F64 ? 8 : 4); }

int check_shape(const qdw_op* op, int prec, int ts, int nt, int pipe, int walk, int march)
{
    QDW_CHECK(!march || march_lds(prec, ts) <= 65536, QDW_EINVAL,
              "D kernel shape: a marching FP64 workgroup of 128 sites per parity needs more "
              "than 64 KB of LDS");
    QDW_CHECK(march == 0 || march == 1, QDW_EINVAL, "D kernel shape: march must be 0 or 1");
    QDW_CHECK(ts == 64 || ts == 128, QDW_EINVAL, "D kernel shape: ts must be 64 or 128");
    QDW_CHECK(nt >= 1 && nt <= 64 && op->g.L[0] % nt == 0, QDW_EINVAL,
              "D kernel shape: nt must divide T and lie in 1..64");
    QDW_CHECK(pipe == 0 || pipe == 1, QDW_EINVAL, "D kernel shape: pipe must be 0 or 1");
    QDW_CHECK(walk == 0 || walk == 1, QDW_EINVAL, "D kernel shape: walk must be 0 or 1");
    return QDW_OK;
}
}  // namespace

extern "C" int qdw_set_dw_shape(qdw_op* op, qdw_prec prec, int ts, int nt, int pipe, int walk,
                                int march)
{
    QDW_CHECK(op, QDW_EINVAL, "qdw_set_dw_shape: null operator");
    QDW_CHECK(prec >= QDW_F64 && prec <= QDW_BF16S, QDW_EINVAL, "qdw_set_dw_shape: bad precision");
    const int rc = check_shape(op, prec, ts, nt, pipe, walk, march);
    if (rc) return rc;
    op->dw_shape[prec] = {ts, nt, pipe, walk, march};
    return QDW_OK;
}

extern "C" int qdw_get_dw_shape(const qdw_op* op, qdw_prec prec, int* shape5)
{
    QDW_CHECK(op && shape5, QDW_EINVAL, "qdw_get_dw_shape: null argument");
    QDW_CHECK(prec >= QDW_F64 && prec <= QDW_BF16S, QDW_EINVAL, "qdw_get_dw_shape: bad precision");
    shape5[0] = op->dw_shape[prec].ts;
    shape5[1] = op->dw_shape[prec].nt;
    shape5[2] = op->dw_shape[prec].pipe;
    shape5[3] = op->dw_shape[prec].walk;
    shape5[4] = op->dw_shape[prec].march;
    return QDW_OK;
}

extern "C" size_t qdw_autotune_workspace_bytes(const qdw_op* op, qdw_prec prec, int nrhs)
{
    if (!op || prec < QDW_F64 || prec > QDW_BF16S || nrhs < 1 || nrhs > kMaxRhs) return 0;
    return 2 * spinor_bytes(op->g, prec) * nrhs + 256;
}

extern "C" int qdw_autotune(qdw_op* op, qdw_prec prec, int nrhs, void* work, size_t work_bytes,
                            char* report, size_t report_len, void* stream)
{
    QDW_CHECK(op, QDW_EINVAL, "qdw_autotune: null operator");
    QDW_CHECK(prec >= QDW_F64 && prec <= QDW_BF16S, QDW_EINVAL, "qdw_autotune: bad precision");
    QDW_CHECK(nrhs >= 1 && nrhs <= kMaxRhs, QDW_EINVAL, "qdw_autotune: need 1 <= nrhs <= 64");
    QDW_CHECK(work, QDW_EINVAL, "qdw_autotune: null workspace");
    QDW_CHECK(work_bytes >= qdw_autotune_workspace_bytes(op, prec, nrhs), QDW_EWORKSPACE,
              "qdw_autotune: workspace smaller than qdw_autotune_workspace_bytes()");
    hipStream_t st = (hipStream_t)stream;
    const Geom& g = op->g;
    const size_t fb = spinor_bytes(g, prec);
    char* buf = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
    RhsTable tab{};
    for (int r = 0; r < nrhs; ++r) {
        tab.in[r] = buf + (size_t)r * fb;
        tab.out[r] = buf + (size_t)(nrhs + r) * fb;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const auto keep = op->dw_shape[prec];
    struct Cand { int ts, nt, pipe, walk, march; float ms; };
    std::vector<Cand> cands;
    for (int march = 0; march < 2; ++march)
        for (int walk = 0; walk < 2; ++walk)
            for (int ts : {64, 128})
                for (int nt = 1; nt <= 64; nt *= 2) {
                    if (g.L[0] % nt) continue;
                    if (march && march_lds(prec, ts) > 65536) continue;
                    for (int pipe = 0; pipe < 2; ++pipe)
                        cands.push_back({ts, nt, pipe, walk, march, 0.f});
                }
    int rc = QDW_OK;
    auto run = [&]() -> int {
        int r0 = fill_pattern(buf, 2 * fb * nrhs, prec, st);
        if (r0) return r0;
        QDW_HIP(hipEventCreate(&e0));
        QDW_HIP(hipEventCreate(&e1));
        for (Cand& c : cands) {
            op->dw_shape[prec] = {c.ts, c.nt, c.pipe, c.walk, c.march};
            int r;
            for (int w = 0; w < 2; ++w)
                if ((r = dispatch(op, tab, nrhs, prec, false, st))) return r;
            const int reps = 8;
            QDW_HIP(hipEventRecord(e0, st));
            for (int w = 0; w < reps; ++w)
                if ((r = dispatch(op, tab, nrhs, prec, false, st))) return r;
            QDW_HIP(hipEventRecord(e1, st));
            QDW_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            QDW_HIP(hipEventElapsedTime(&ms, e0, e1));
            c.ms = ms / reps;
        }
        return QDW_OK;
    };
    rc = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    if (rc) {
        op->dw_shape[prec] = keep;
        return rc;
    }
    const Cand* best = &cands[0];
    for (const Cand& c : cands)
        if (c.ms < best->ms) best = &c;
    op->dw_shape[prec] = {best->ts, best->nt, best->pipe, best->walk, best->march};
    if (report && report_len) {
        std::string s;
        char line[200];
        std::snprintf(line, sizeof line,
                      "lattice %dx%dx%dx%d prec %d nrhs %d: best ts=%d nt=%d pipe=%d walk=%d march=%d %.4f ms;",
                      g.L[0], g.L[1], g.L[2], g.L[3], (int)prec, nrhs, best->ts, best->nt,
                      best->pipe, best->walk, best->march, best->ms);
        s += line;
        for (const Cand& c : cands) {
            std::snprintf(line, sizeof line, " [%d,%d,%d,%d,%d]=%.4f", c.ts, c.nt, c.pipe, c.walk,
                          c.march, c.ms);
            s += line;
        }
        std::snprintf(report, report_len, "%s", s.c_str());
    }
    return QDW_OK;
}
