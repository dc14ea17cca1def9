// nn.hip -- a learned gauge-covariant preconditioner for flexible GCR (not from the paper;
// the paper's solvers tolerate any preconditioner that changes from step to step).
//
// Network: three linear parallel-transport layers with 1 -> 8 -> 8 -> 1 spinor channels.
// A layer maps channels in_b to
//     out_a(x) = sum_{p=0..8} sum_b W_p[a][b] (T_p in_b)(x)
// with T_0 = 1, T_{+mu} v(x) = s U_mu(x) v(x+mu), T_{-mu} v(x) = s U_mu(x-mu)^+ v(x-mu)
// (s the fermion boundary sign) and W_p[a][b] a complex 4x4 matrix acting on spin only,
// so the network commutes with gauge transformations.
//
// GPU mapping of a layer: (1) a transport kernel writes, for every site x and colour c,
// one row of the matrix A[(x, c)][(p, b, t, re/im)] (t a spin index), stored in panels of
// eight columns (one (p, b) group per panel, so each lane writes contiguous runs and
// consecutive lanes write consecutive runs); (2) the channel
// mixing is the real GEMM out[(x, c)][(a, s, re/im)] = A B with B the real embedding of the
// complex weights, run on the matrix cores: bf16 operands and FP32 accumulation
// (v_mfma_f32_16x16x16_bf16), or FP32 operands (v_mfma_f32_16x16x4_f32) for gradient
// checks. Backward: dA = G B^T (matrix cores), then the adjoint transport gathers dA back
// to the input channels; dB = A^T G (matrix cores, split over rows, fixed-order reduction)
// gives the weight gradient. Adam updates FP32 master weights.
#include <cmath>
#include <vector>

#include "blas.h"
#include "dirac_core.h"

namespace qdw {

namespace {

constexpr int kPaths = 9;
constexpr int kLayers = 3;
constexpr int kCh[kLayers + 1] = {1, 8, 8, 1};
constexpr int kMaxK = 72 * 8;   // 9 paths x 8 channels x 4 spins x 2
constexpr int kMaxN = 64;       // 8 channels x 4 spins x 2

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

inline int layer_K(int l) { return (kPaths * kCh[l] * 8 + 15) & ~15; }
inline int layer_N(int l) { return std::max(16, kCh[l + 1] * 8); }
inline int layer_w_offset(int l)  // in complex numbers
{
    int o = 0;
    for (int j = 0; j < l; ++j) o += kPaths * kCh[j] * kCh[j + 1] * 16;
    return o;
}
inline int total_weights() { return layer_w_offset(kLayers); }

inline long rows_of(const Geom& g) { return (long)2 * padded(g.Vh) * 3; }
inline long rows_padded(const Geom& g) { return (rows_of(g) + 63) & ~63L; }

// A and dA in panels of 8 columns: element (row m, column k) of a matrix with Mp rows
__device__ __forceinline__ long pidx(long Mp, long m, int k)
{
    return (((long)(k >> 3) * Mp + m) << 3) + (k & 7);
}

// two FP32 values rounded to bf16 (to nearest even, by the conversion instruction) and
// packed into one register, lo in the low half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi)
{
    const bf16x2_t b = __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t);
    uint32_t r;
    __builtin_memcpy(&r, &b, 4);
    return r;
}

// 8 consecutive values of one panel row
template <bool F32M>
__device__ __forceinline__ void put8(void* A, long at, const float v[8])
{
    if constexpr (F32M) {
        float4* d = (float4*)((float*)A + at);
        d[0] = make_float4(v[0], v[1], v[2], v[3]);
        d[1] = make_float4(v[4], v[5], v[6], v[7]);
    } else {
        uint4 r;
        r.x = pack_bf16x2(v[0], v[1]);
        r.y = pack_bf16x2(v[2], v[3]);
        r.z = pack_bf16x2(v[4], v[5]);
        r.w = pack_bf16x2(v[6], v[7]);
        *(uint4*)((uint16_t*)A + at) = r;
    }
}

__device__ __forceinline__ uint16_t bf16_bits(float f) { return float_to_bf16(f); }

template <bool F32M>
__device__ __forceinline__ void put_el(void* A, long at, float v)
{
    if (F32M) ((float*)A)[at] = v;
    else ((uint16_t*)A)[at] = bf16_bits(v);
}

// one complex component (spin s, colour c) of an FP32 eo-SoA field at site (par, i)
__device__ __forceinline__ long f32_addr(int Vh, int par, int i, int s, int c)
{
    const int k12 = s * 3 + c;
    return chunk_at(Vh, 6, par, k12 >> 1, i) * 4 + (k12 & 1) * 2;
}

// ------------------------------------------------------------------ transport
//
// A[(q, c)][((p*Cin + b)*4 + t)*2 + re/im] = (T_p in_b)(q)[t][c], q = par*Vp + i. Rows of
// padded sites and the padding columns K..Kpad-1 are written as zeros, so the matrix holds
// no stale values from earlier use of the workspace.
template <bool F32M, int PIN>
__global__ __launch_bounds__(256) void nn_transport_kernel(Geom g, int Cin, int Kpad, long Mp,
                                                           const void* const* in, void* A,
                                                           const void* links, const void* dets)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int Vp = padded(g.Vh);
    const long nq = 2L * Vp;
    if (tid >= nq * Cin) return;
    const int b = (int)(tid / nq);
    const long q = tid - (long)b * nq;
    const int par = (int)(q / Vp), i = (int)(q - (long)par * Vp);
    const float zero[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (b == Cin - 1)
        for (int kg = kPaths * Cin; kg < Kpad / 8; ++kg)
            for (int c = 0; c < 3; ++c) put8<F32M>(A, pidx(Mp, q * 3 + c, kg * 8), zero);
    if (i >= g.Vh) {
        for (int p = 0; p < kPaths; ++p)
            for (int c = 0; c < 3; ++c) put8<F32M>(A, pidx(Mp, q * 3 + c, (p * Cin + b) * 8), zero);
        return;
    }
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const void* v = in[b];
    for (int p = 0; p < kPaths; ++p) {
        cx<float> s[12], w[12];
        if (p == 0) {
            load_spinor<PIN>(v, g.Vh, par, i, s);
            for (int k = 0; k < 12; ++k) w[k] = s[k];
        } else {
            const int mu = (p - 1) >> 1;
            const bool fwd = ((p - 1) & 1) == 0;
            const int j = (fwd ? lex_fwd(g, x, lex, mu) : lex_bwd(g, x, lex, mu)) >> 1;
            load_spinor<PIN>(v, g.Vh, 1 - par, j, s);
            cx<float> u[6], d;
            float sg = 1.f;
            if (fwd) {
                load_link<F32>(links, dets, g.Vh, par, i, mu, u, d);
                if (mu == 0 && x[0] == g.L[0] - 1) sg = (float)g.bc_t;
            } else {
                load_link<F32>(links, dets, g.Vh, 1 - par, j, mu, u, d);
                if (mu == 0 && x[0] == 0) sg = (float)g.bc_t;
            }
            // the SU(3) multiply of dirac_core acts on two spin components at a time
            cx<float> h[6], o[6];
            for (int half = 0; half < 2; ++half) {
                for (int k = 0; k < 6; ++k) h[k] = scale(s[6 * half + k], sg);
                if (fwd) su3_mul<float, false>(u, d, h, o);
                else su3_mul<float, true>(u, d, h, o);
                for (int k = 0; k < 6; ++k) w[6 * half + k] = o[k];
            }
        }
        // rows (q, c): 8 consecutive entries (t, re/im) of the (p, b) panel
        const int k0 = (p * Cin + b) * 8;
        for (int c = 0; c < 3; ++c) {
            float v[8];
            for (int t = 0; t < 4; ++t) {
                v[2 * t] = w[t * 3 + c].re;
                v[2 * t + 1] = w[t * 3 + c].im;
            }
            put8<F32M>(A, pidx(Mp, q * 3 + c, k0), v);
        }
    }
}

// g_b(x) = sum_p T_p^+ dA[p][b](x): T_{+mu}^+ = T_{-mu}, T_{-mu}^+ = T_{+mu}
__global__ __launch_bounds__(256) void nn_transport_adj_kernel(Geom g, int Cin, long Mp,
                                                               const float* dA, float* const* gout,
                                                               const void* links, const void* dets)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int Vp = padded(g.Vh);
    const long nq = 2L * Vp;
    if (tid >= nq * Cin) return;
    const int b = (int)(tid / nq);
    const long q = tid - (long)b * nq;
    const int par = (int)(q / Vp), i = (int)(q - (long)par * Vp);
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<float> acc[12];
    auto rows = [&](long qq, int p, cx<float> w[12]) {
        const int k0 = (p * Cin + b) * 8;
        for (int c = 0; c < 3; ++c) {
            const float4* r = (const float4*)(dA + pidx(Mp, qq * 3 + c, k0));
            const float4 lo = r[0], hi = r[1];
            w[c] = {lo.x, lo.y};
            w[3 + c] = {lo.z, lo.w};
            w[6 + c] = {hi.x, hi.y};
            w[9 + c] = {hi.z, hi.w};
        }
    };
    rows(q, 0, acc);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = 0; dir < 2; ++dir) {
            // dir 0: the +mu path of site y = x - mu lands here through U_mu(y)^+
            // dir 1: the -mu path of site y = x + mu lands here through U_mu(x)
            const bool from_below = dir == 0;
            const int ylex = from_below ? lex_bwd(g, x, lex, mu) : lex_fwd(g, x, lex, mu);
            const long yq = (long)(1 - par) * Vp + (ylex >> 1);
            cx<float> w[12], u[6], d, h[6], o[6];
            rows(yq, from_below ? 1 + 2 * mu : 2 + 2 * mu, w);
            float sg = 1.f;
            if (from_below) {
                load_link<F32>(links, dets, g.Vh, 1 - par, ylex >> 1, mu, u, d);
                if (mu == 0 && x[0] == 0) sg = (float)g.bc_t;
            } else {
                load_link<F32>(links, dets, g.Vh, par, i, mu, u, d);
                if (mu == 0 && x[0] == g.L[0] - 1) sg = (float)g.bc_t;
            }
            for (int half = 0; half < 2; ++half) {
                for (int k = 0; k < 6; ++k) h[k] = scale(w[6 * half + k], sg);
                if (from_below) su3_mul<float, true>(u, d, h, o);
                else su3_mul<float, false>(u, d, h, o);
                for (int k = 0; k < 6; ++k) acc[6 * half + k] = acc[6 * half + k] + o[k];
            }
        }
    }
    store_spinor<F32>(gout[b], g.Vh, par, i, acc);
}

// ------------------------------------------------------------------ weights as matrices
//
// Real embedding of the complex weights, B[k][n] with k = ((p*Cin + b)*4 + t)*2 + ri,
// n = (a*4 + s)*2 + ro: B[(.., re)][(.., re)] = Re W, B[(.., im)][(.., re)] = -Im W,
// B[(.., re)][(.., im)] = Im W, B[(.., im)][(.., im)] = Re W, W = W_p[a][b][s][t].
// Stored transposed, Bt[n][k], for the forward GEMM, and as Bk[k][n] for dA = G B^T.
__device__ __forceinline__ float embed(const float* W, int Cin, int Cout, int k, int n)
{
    const int ri = k & 1, kk = k >> 1, t = kk & 3, pb = kk >> 2, b = pb % Cin, p = pb / Cin;
    const int ro = n & 1, nn = n >> 1, s = nn & 3, a = nn >> 2;
    if (a >= Cout || p >= kPaths) return 0.f;
    const long w = ((((long)p * Cout + a) * Cin + b) * 4 + s) * 4 + t;
    const float re = W[2 * w], im = W[2 * w + 1];
    if (ro == 0) return ri == 0 ? re : -im;
    return ri == 0 ? im : re;
}

template <bool F32M>
__global__ void nn_embed_kernel(const float* W, int Cin, int Cout, int Kpad, int Npad, void* Bt,
                                void* Bk)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= Kpad * Npad) return;
    const int n = tid / Kpad, k = tid - n * Kpad;
    const float v = (k < kPaths * Cin * 8) ? embed(W, Cin, Cout, k, n) : 0.f;
    put_el<F32M>(Bt, (long)n * Kpad + k, v);
    put_el<F32M>(Bk, (long)k * Npad + n, v);
}

// dW (complex, dL/dRe W + i dL/dIm W) += the real-embedding gradient dB[k][n]
__global__ void nn_dw_kernel(const float* dB, int Cin, int Cout, int Npad, float* dW)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = kPaths * Cout * Cin * 16;
    if (tid >= nw) return;
    const int t = tid & 3, s = (tid >> 2) & 3, rest = tid >> 4;
    const int b = rest % Cin, a = (rest / Cin) % Cout, p = rest / (Cin * Cout);
    const int kr = (((p * Cin + b) * 4 + t) * 2), nr = ((a * 4 + s) * 2);
    const float d_rr = dB[(long)kr * Npad + nr], d_ii = dB[(long)(kr + 1) * Npad + nr + 1];
    const float d_ir = dB[(long)(kr + 1) * Npad + nr], d_ri = dB[(long)kr * Npad + nr + 1];
    dW[2 * tid] += d_rr + d_ii;
    dW[2 * tid + 1] += d_ri - d_ir;
}

// ------------------------------------------------------------------ GEMMs on matrix cores

// acc[j] += A[m0 : m0+16][k0 : k0+KS] * B[k0 : k0+KS][16 j : 16 j + 16] for one wave;
// A row-major (element (m, k) at arow + k for this lane's row) or, with Mp > 0, in panels
template <bool F32M>
__device__ __forceinline__ void mfma_step(const void* A, long arow, const void* Bt, long brow0,
                                          long bstride, int kofs, int nt, f4 acc[4], long Mp = 0,
                                          long row = 0)
{
    const long ai = Mp > 0 ? pidx(Mp, row, kofs) : arow + kofs;
    if constexpr (!F32M) {
        const s4 a = *(const s4*)((const uint16_t*)A + ai);
        for (int j = 0; j < nt; ++j) {
            const s4 b = *(const s4*)((const uint16_t*)Bt + brow0 + j * 16 * bstride + kofs);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
        }
    } else {
        const float a = ((const float*)A)[ai];
        for (int j = 0; j < nt; ++j) {
            const float b = ((const float*)Bt)[brow0 + j * 16 * bstride + kofs];
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
        }
    }
}

// out channels (FP32 fields) = A Bt^T; a workgroup computes 64 rows, a wave 16 rows x Npad
template <bool F32M>
__global__ __launch_bounds__(256) void nn_gemm_out_kernel(Geom g, int Kpad, int Npad, int Cout,
                                                          long Mp, const void* A, const void* Bt,
                                                          float* const* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long m0 = (long)blockIdx.x * 64 + wave * 16;
    const int nt = Npad / 16;
    f4 acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    const int KS = F32M ? 4 : 16;
    const long row = m0 + (lane & 15);
    const long brow0 = (long)(lane & 15) * Kpad;
    const int kl = F32M ? (lane >> 4) : 4 * (lane >> 4);
    for (int k0 = 0; k0 < Kpad; k0 += KS)
        mfma_step<F32M>(A, 0, Bt, brow0, Kpad, k0 + kl, nt, acc, Mp, row);
    const int Vp = padded(g.Vh);
    for (int j = 0; j < nt; ++j)
        for (int r = 0; r < 4; ++r) {
            const long m = m0 + 4 * (lane >> 4) + r;
            const int n = j * 16 + (lane & 15);
            const long q = m / 3;
            const int c = (int)(m - q * 3);
            const int a = n >> 3, s = (n >> 1) & 3, ri = n & 1;
            if (q >= 2L * Vp || a >= Cout) continue;
            const int par = (int)(q / Vp), i = (int)(q - (long)par * Vp);
            if (i >= g.Vh) continue;
            out[a][f32_addr(g.Vh, par, i, s, c) + ri] = acc[j][r];
        }
}

// dA[m][k] = sum_n G[m][n] Bk[k][n]  (G = gradient of the layer output, FP32 rows)
template <bool F32M>
__global__ __launch_bounds__(256) void nn_gemm_da_kernel(int Kpad, int Npad, long Mp, const void* G,
                                                         const void* Bk, float* dA)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long m0 = (long)blockIdx.x * 64 + wave * 16;
    const int KS = F32M ? 4 : 16;
    const long arow = (m0 + (lane & 15)) * Npad;
    const int kl = F32M ? (lane >> 4) : 4 * (lane >> 4);
    for (int kt = 0; kt < Kpad / 16; kt += 4) {
        const int nt = std::min(4, Kpad / 16 - kt);
        f4 acc[4];
        for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
        const long brow0 = (long)(kt * 16 + (lane & 15)) * Npad;
        for (int n0 = 0; n0 < Npad; n0 += KS)
            mfma_step<F32M>(G, arow, Bk, brow0, Npad, n0 + kl, nt, acc);
        for (int j = 0; j < nt; ++j)
            for (int r = 0; r < 4; ++r)
                dA[pidx(Mp, m0 + 4 * (lane >> 4) + r, (kt + j) * 16 + (lane & 15))] = acc[j][r];
    }
}

// partial dB[k][n] over a slice of rows: D[k][n] += sum_m A[m][k] G[m][n]
template <bool F32M>
__global__ __launch_bounds__(256) void nn_gemm_db_kernel(long M, int Kpad, int Npad, int rows_per,
                                                         long Mp, const void* A, const void* G,
                                                         float* part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kt = blockIdx.x;     // 16 columns k of A
    const int split = blockIdx.y;  // slice of rows
    const int nt = Npad / 16;
    if (wave >= nt) return;
    const long mbeg = (long)split * rows_per;
    const long mend = std::min(M, mbeg + rows_per);
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    const int kcol = kt * 16 + (lane & 15);
    const int ncol = wave * 16 + (lane & 15);
    if constexpr (!F32M) {
        const uint16_t* Au = (const uint16_t*)A;
        const uint16_t* Gu = (const uint16_t*)G;
        for (long m = mbeg; m < mend; m += 16) {
            s4 a, b;
            for (int j = 0; j < 4; ++j) {
                const long mm = m + 4 * (lane >> 4) + j;
                a[j] = (short)Au[pidx(Mp, mm, kcol)];
                b[j] = (short)Gu[mm * Npad + ncol];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
    } else {
        const float* Af = (const float*)A;
        const float* Gf = (const float*)G;
        for (long m = mbeg; m < mend; m += 4) {
            const long mm = m + (lane >> 4);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[pidx(Mp, mm, kcol)], Gf[mm * Npad + ncol],
                                                        acc, 0, 0, 0);
        }
    }
    for (int r = 0; r < 4; ++r) {
        const int k = kt * 16 + 4 * (lane >> 4) + r;
        part[((long)split * Kpad + k) * Npad + ncol] = acc[r];
    }
}

__global__ void nn_reduce_db_kernel(const float* part, int nsplit, int KN, float* dB)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= KN) return;
    float s = 0.f;
    for (int p = 0; p < nsplit; ++p) s += part[(long)p * KN + tid];
    dB[tid] = s;
}

// G rows from a channel gradient (FP32 fields), times `scale`
template <bool F32M>
__global__ __launch_bounds__(256) void nn_pack_g_kernel(Geom g, int Cout, int Npad,
                                                        const float* const* gf, float scale, void* G)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int Vp = padded(g.Vh);
    const long nq = 2L * Vp;
    if (tid >= nq) return;
    const int par = (int)(tid / Vp), i = (int)(tid - (long)par * Vp);
    for (int c = 0; c < 3; ++c)
        for (int n = 0; n < Npad; ++n) {
            const int a = n >> 3, s = (n >> 1) & 3, ri = n & 1;
            float v = 0.f;
            if (a < Cout && i < g.Vh) v = scale * gf[a][f32_addr(g.Vh, par, i, s, c) + ri];
            put_el<F32M>(G, (tid * 3 + c) * Npad + n, v);
        }
}

// ------------------------------------------------------------------ fused forward layer
//
// The production forward pass (bf16 operands) fuses transport and mixing: a workgroup
// owns 64 consecutive sites q (192 rows (q, c)); for each batch of paths (one path when
// Cin = 8, all nine when Cin = 1) its lanes transport the input channels into the rows'
// columns for that batch, then the four wavefronts multiply them by the batch's rows of B
// on the matrix cores, 48 rows each, accumulating in FP32 -- with Cin = 1 through an LDS
// tile (the waves share the paths), with Cin = 8 straight from the registers the
// transports leave (each wave transports the 16 sites whose rows it multiplies). Columns
// are visited in the same order as by the unfused kernels, so both give the same sums; the
// difference is that A never goes to HBM. A lane always transports for the same site: its
// coordinates are computed once, and with Cin = 8 one link load serves the lane's two
// channels.

// neighbour index, boundary sign and link of path p (1..8) at site (par, i)
__device__ __forceinline__ void nn_path_setup(const Geom& g, int par, int i, const int x[4], int lex,
                                              int p, const void* links, const void* dets, int& j,
                                              float& sg, cx<float> u[6], cx<float>& d)
{
    const int mu = (p - 1) >> 1;
    const bool fwd = ((p - 1) & 1) == 0;
    j = (fwd ? lex_fwd(g, x, lex, mu) : lex_bwd(g, x, lex, mu)) >> 1;
    sg = 1.f;
    if (fwd) {
        load_link<F32>(links, dets, g.Vh, par, i, mu, u, d);
        if (mu == 0 && x[0] == g.L[0] - 1) sg = (float)g.bc_t;
    } else {
        load_link<F32>(links, dets, g.Vh, 1 - par, j, mu, u, d);
        if (mu == 0 && x[0] == 0) sg = (float)g.bc_t;
    }
}

// the 3x3 matrix s U of a path's link, its third row rebuilt once (s = +-1, so folding it
// into the matrix changes no rounding)
__device__ __forceinline__ void nn_link_matrix(const cx<float> u[6], cx<float> d, float sg,
                                               cx<float> m[9])
{
    m[6] = d * conj_(cmadd(u[1] * u[5], -u[2], u[4]));
    m[7] = d * conj_(cmadd(u[2] * u[3], -u[0], u[5]));
    m[8] = d * conj_(cmadd(u[0] * u[4], -u[1], u[3]));
#pragma unroll
    for (int k = 0; k < 6; ++k) m[k] = u[k];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = scale(m[k], sg);
}

// A path's link matrix as bf16 pairs for the dot-product instruction that multiplies two
// bf16 pairs and adds both products to an FP32 sum (v_dot2_f32_bf16): the hidden channels are
// stored as (re, im) bf16 pairs, so with a = (e.re, -e.im), b = (e.im, e.re) one complex
// product e v adds dot(a, v) to the real and dot(b, v) to the imaginary part -- two
// instructions instead of four FMAs, and no widening of the stored spinor. Entry r * 3 + k is
// the coefficient of v_k in w_r: M[r][k] for a forward path, conj(M[k][r]) for a backward one.
// The link is rounded to bf16 like the operands of the mixing that follows.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
struct LinkBF {
    uint32_t a[9], b[9];
};

__device__ __forceinline__ void nn_link_bf16(bool fwd, const cx<float> m[9], LinkBF& L)
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const cx<float> e = fwd ? m[3 * r + k] : conj_(m[3 * k + r]);
            L.a[3 * r + k] = pack_bf16x2(e.re, -e.im);
            L.b[3 * r + k] = pack_bf16x2(e.im, e.re);
        }
}

__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c)
{
    bf16x2v x, y;
    __builtin_memcpy(&x, &a, 4);
    __builtin_memcpy(&y, &b, 4);
    return __builtin_amdgcn_fdot2_f32_bf16(x, y, c, false);
}

// w = (M or M^+) v (ACC: w += ...) for the four spins of a spinor stored as 12 (re, im)
// bf16 pairs (three 16-byte chunks as loaded), FP32 sums
template <bool ACC = false>
__device__ __forceinline__ void nn_transport_dot2(const LinkBF& L, const u32x4 raw[3], cx<float> w[12])
{
    uint32_t v[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[4 * k] = raw[k].x;
        v[4 * k + 1] = raw[k].y;
        v[4 * k + 2] = raw[k].z;
        v[4 * k + 3] = raw[k].w;
    }
#pragma unroll
    for (int sd = 0; sd < 4; ++sd)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            float re = ACC ? w[3 * sd + r].re : 0.f, im = ACC ? w[3 * sd + r].im : 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                re = dot2_bf16(L.a[3 * r + k], v[3 * sd + k], re);
                im = dot2_bf16(L.b[3 * r + k], v[3 * sd + k], im);
            }
            w[3 * sd + r] = {re, im};
        }
}

// w = M sp (forward path) or M^+ sp (backward path) for the four spins
__device__ __forceinline__ void nn_apply_m(bool fwd, const cx<float> m[9], const cx<float> sp[12],
                                           cx<float> w[12])
{
#pragma unroll
    for (int sd = 0; sd < 4; ++sd) {
        const cx<float> h0 = sp[3 * sd], h1 = sp[3 * sd + 1], h2 = sp[3 * sd + 2];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            w[3 * sd + r] = fwd ? cmadd(cmadd(m[3 * r] * h0, m[3 * r + 1], h1), m[3 * r + 2], h2)
                                : cmadd_conj(cmadd_conj(cmul_conj(m[r], h0), m[3 + r], h1),
                                             m[6 + r], h2);
    }
}

// one path's 64 x 64 block of the 8-channel layer's weights (bf16), as the fused kernel
// keeps it in LDS
constexpr int kWBlock = 64 * 64 * 2;
typedef __attribute__((address_space(1))) const u32x4 g_cu4;

// the 8-channel layer's weights in the fused kernel's LDS image: for each path p the block
// of Bt (rows n < 64, columns k = 64 p + 0..63) as [k / 4][n][k % 4], so that one lane's
// four consecutive k of one column n are 8 contiguous bytes and the 16 lanes of a
// matrix-core operand row read 128 contiguous bytes
__global__ void nn_embed_lds_kernel(const uint16_t* Bt, int Kpad, uint16_t* Bl)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= kPaths * 64 * 64) return;
    const int e = tid & 7, n = (tid >> 3) & 63, kq = (tid >> 9) & 7, p = tid >> 12;
    Bl[tid] = Bt[(long)n * Kpad + p * 64 + kq * 8 + e];
}

// LDS row stride (in bf16 halves) of a tile with KB columns: at least KB + 8, rows 16-byte
// aligned, and a lane's three rows (the lane-to-lane step of the 16-byte row writes) 4 banks
// apart modulo the 64 banks, so the 64 lanes of a write hit every bank equally
constexpr int tile_stride(int kb)
{
    int ls = (kb + 8 + 7) / 8 * 8;
    while ((3 * ls / 2) % 64 != 4) ls += 8;
    return ls;
}

// first row q (site) of the 64-site block of this workgroup in the forward kernels, whose
// grid is one workgroup per block of either parity: blocks of the two parities alternate
// (the even and odd sites of one index range are lexicographic neighbours along x3), and
// each XCD takes one contiguous range of blocks, so that the neighbour windows a workgroup
// gathers were mostly loaded into its XCD's L2 by workgroups running beside it
__device__ __forceinline__ long nn_block_q0(int Vp)
{
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    return (long)(w & 1) * Vp + (long)(w >> 1) * 64;
}

// the three rows (site sl, colour c) of one (path, channel) group, as bf16, into the tile
template <int LS>
__device__ __forceinline__ void nn_put_rows(uint16_t* tile, int sl, int k0, const cx<float> w[12])
{
    for (int c = 0; c < 3; ++c) {
        uint4 r;
        r.x = pack_bf16x2(w[c].re, w[c].im);
        r.y = pack_bf16x2(w[3 + c].re, w[3 + c].im);
        r.z = pack_bf16x2(w[6 + c].re, w[6 + c].im);
        r.w = pack_bf16x2(w[9 + c].re, w[9 + c].im);
        *(uint4*)&tile[(sl * 3 + c) * LS + k0] = r;
    }
}

// the same rows as the matrix-core operands of colours 0..2: (re, im) of spins 0..3 as bf16
// (the eight columns of one channel that a lane supplies for its site)
__device__ __forceinline__ void nn_rows(const cx<float> w[12], bf16x8 T[3])
{
    for (int c = 0; c < 3; ++c) {
        const uint32_t v[4] = {pack_bf16x2(w[c].re, w[c].im), pack_bf16x2(w[3 + c].re, w[3 + c].im),
                               pack_bf16x2(w[6 + c].re, w[6 + c].im), pack_bf16x2(w[9 + c].re, w[9 + c].im)};
        __builtin_memcpy(&T[c], v, 16);
    }
}

// the same straight from a spinor stored as bf16 pairs (the identity path)
__device__ __forceinline__ void nn_rows_raw(const u32x4 raw[3], bf16x8 T[3])
{
    uint32_t v[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[4 * k] = raw[k].x;
        v[4 * k + 1] = raw[k].y;
        v[4 * k + 2] = raw[k].z;
        v[4 * k + 3] = raw[k].w;
    }
    for (int c = 0; c < 3; ++c) {
        const uint32_t t[4] = {v[c], v[3 + c], v[6 + c], v[9 + c]};
        __builtin_memcpy(&T[c], t, 16);
    }
}

// MIXOUT (inference passes of the 8 -> 8 layer only): instead of storing the layer's eight
// output channels, the kernel goes on with the last layer's path mixing on them (the
// product nn_mix_paths_kernel forms, with the mixing matrix Bm) and stores the nine m_p
// fields to out[0..8]; its operand is the outputs rounded to bf16, as the stored hidden
// channels would be, taken from the registers that hold them, and the products sum over
// the same K steps in the same order (the forward pass's output at 32^3 x 64 was checked
// bit for bit against the two-kernel form).
// Occupancy: the one-channel layer is held to 128 registers, four waves per SIMD, where its
// gathers (two or three paths per wave, one after the other) hide behind the other waves
// (the compiler's own choice, 132, allows three); the eight-channel layers keep theirs.
template <int CIN, int COUT, int PIN, int POUT, bool MIXOUT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CIN == 1 ? 4 : 1)))
void nn_layer_fused_kernel(Geom g, int Kpad, const void* const* in, const void* Bt,
                           const void* Bl, void* const* out, const void* links,
                           const void* dets, const uint16_t* Bm = nullptr)
{
    constexpr int PB = CIN == 1 ? kPaths : 1;          // paths per batch
    constexpr int KB = (PB * CIN * 8 + 15) & ~15;      // columns per batch (80 or 64)
    constexpr int LS = tile_stride(KB);                // LDS row stride (halves)
    constexpr int NT = COUT * 8 >= 16 ? COUT * 8 / 16 : 1;  // 16-column tiles of N
    static_assert(CIN == 1 || CIN == 8, "channel counts of the network");
    static_assert(CIN == 1 || (KB == 64 && NT == 4), "the LDS weight image is a 64 x 64 block");
    // LDS: Cin = 1, the transported tile of the batch; Cin = 8, two 8 KiB buffers for the
    // weight blocks of the current and the next path (its transports go to the matrix
    // cores from the registers); then the output block (COUT channels x 24 reals x 64
    // sites, bf16)
    constexpr int TILE_B = CIN == 1 ? 192 * LS * 2 : 0, W_B = CIN == 8 ? 2 * kWBlock : 0;
    // output staging in bf16: one row per (channel, 16-byte chunk) of 64 sites x 8 halves,
    // padded by one chunk so that consecutive rows start 4 banks apart
    static_assert(POUT == BF16S, "the layers' outputs are bf16 hidden channels");
    constexpr int OROW = 64 * 8 + 8;
    constexpr int OUT_B = (MIXOUT ? kPaths : COUT) * 3 * OROW * 2;
    static_assert(!MIXOUT || (CIN == 8 && COUT == 8), "the path mixing follows the 8 -> 8 layer");
    static_assert(TILE_B % 16 == 0, "weight blocks 16-byte aligned");
    __shared__ __attribute__((aligned(16))) char lds[TILE_B + W_B > OUT_B ? TILE_B + W_B : OUT_B];
    uint16_t* tile = (uint16_t*)lds;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // Cin = 8: the weight block of path p is in buffer p & 1, as [k/8][n][k%8] (bf16)
    uint16_t* const wbuf = (uint16_t*)(lds + TILE_B);
    const uint16_t* wb = wbuf;
    // the site (0..63) and colour of output row 16 r + i (i < 16) of a wave's 48 rows:
    // Cin = 1, the tile's rows 3 site + colour; Cin = 8, colour-major (row tile r is colour
    // r of the wave's 16 sites), the order in which its transports reach the matrix cores
    auto row_site = [&](int r, int i, int& site, int& c) {
        if constexpr (CIN == 8) {
            site = wave * 16 + i;
            c = r;
        } else {
            const int m = wave * 48 + r * 16 + i;
            site = m / 3;
            c = m - site * 3;
        }
    };
    const int Vp = padded(g.Vh);
    const long q0 = nn_block_q0(Vp);
    // this lane's transport site: Cin = 8, the wave's own 16 sites, four lanes per site,
    // channels cg and cg + 4 per lane, so that a lane's transports are the very operand
    // registers it supplies to the wave's products (no LDS between them, and the workgroup
    // meets once per path only, for the shared weight block); Cin = 1, all 64 sites, paths
    // split over the waves
    const int sl = CIN == 8 ? wave * 16 + (lane & 15) : lane;
    const int cg = lane >> 4;
    const long qs = q0 + sl;
    const int par = (int)(qs / Vp), i = (int)(qs - (long)par * Vp);
    const bool real = i < g.Vh;
    int x[4] = {0, 0, 0, 0}, lex = 0;
    if (real) eo_coords(g, par, i, x, lex);
    const cx<float> zero12[12] = {};
    static_assert(CIN == 1 || PIN == BF16S, "hidden channels are stored in bf16");
    f4 acc[3][NT];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < NT; ++j) acc[r][j] = f4{0.f, 0.f, 0.f, 0.f};
    // The products are formed transposed, B^T A^T (the weights as the first operand, the
    // transported rows as the second; the operand registers are the same as for A B):
    // acc[r][j] then holds, in lane l, output row 16 r + l % 16 of the wave's 48 and the
    // four columns 16 j + 4 (l / 16) + e, e = 0..3 -- the layout in which a 16x16x16
    // product takes its operands, so the last layer's mixing reads them from the
    // registers, and consecutive (re, im) columns pair up for 4-byte stores.
    // Cin = 1: rows 48*wave .. +48 of the tile times B[0 .. KB][0 .. 16 NT]
    auto mix_tile = [&]() {
        for (int kk = 0; kk < KB; kk += 16) {
            const int kl = kk + 4 * (lane >> 4);
            s4 bf[NT];
            for (int j = 0; j < NT; ++j)
                bf[j] = *(const s4*)((const uint16_t*)Bt + (long)(j * 16 + (lane & 15)) * Kpad + kl);
            for (int r = 0; r < 3; ++r) {
                const s4 a = *(const s4*)&tile[(wave * 48 + r * 16 + (lane & 15)) * LS + kl];
                for (int j = 0; j < NT; ++j)
                    acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf[j], a, acc[r][j], 0, 0, 0);
            }
        }
    };
    if constexpr (CIN == 8) {
        // The inputs of one path for this lane -- the neighbour spinors of its two channels
        // as stored (bf16, widened when used), the link and the path's weight block -- are
        // loaded ahead of their use: the spinors two paths ahead (three stages), the link and
        // the weights one path ahead (two stages), so the gathered spinors have two paths'
        // transports and products to arrive in. Within one path the weights are issued
        // first, the link next and the spinors last: loads complete in issue order, so the
        // wait for the weights before the path's barrier leaves the link and spinor loads
        // in flight. The stages rotate by name (no indexed arrays).
        struct SpStage {
            u32x4 s0[3], s1[3];
        };
        struct LkStage {
            cx<float> u[6], d;
            float sg;
        };
        // the lane's two channel fields, read from the pointer table once and accessed as
        // global memory: loads through generic pointers would be flat loads, which may
        // complete out of order with the LDS accesses, so that every wait in the path loop
        // would become a wait for all loads in flight, the prefetched ones included
        const g_cu4* const c0 = (const g_cu4*)in[cg];
        const g_cu4* const c1 = (const g_cu4*)in[cg + 4];
        // the spinors of path p: the lane's own site for p = 0, else the neighbour
        auto fetch_sp = [&](int p, SpStage& S) {
            int j = i, pp = par;
            if (p > 0) {
                const int mu = (p - 1) >> 1;
                j = ((((p - 1) & 1) == 0) ? lex_fwd(g, x, lex, mu) : lex_bwd(g, x, lex, mu)) >> 1;
                pp = 1 - par;
            }
            const long b0 = chunk_at(g.Vh, 3, pp, 0, j);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                S.s0[k] = c0[b0 + (long)k * kSB];
                S.s1[k] = c1[b0 + (long)k * kSB];
            }
        };
        // the link and boundary sign of path p (1..8)
        auto fetch_lk = [&](int p, LkStage& L) {
            int j;
            nn_path_setup(g, par, i, x, lex, p, links, dets, j, L.sg, L.u, L.d);
        };
        // the weight block of path p: each of the 256 lanes loads 32 contiguous bytes of it
        // and stores them into the block's LDS buffer once the path before it is done (one
        // workgroup barrier per path; the loads stay in registers meanwhile, in flight
        // during the transport and the matrix-core step)
        const int tid = threadIdx.x;
        auto load_w = [&](int p, u32x4 r[2]) {
            const g_cu4* src = (const g_cu4*)((const char*)Bl + (long)p * kWBlock) + 2 * tid;
            r[0] = src[0];
            r[1] = src[1];
        };
        auto store_w = [&](int p, const u32x4 r[2]) {
            u32x4* dst = (u32x4*)((char*)wbuf + (p & 1) * kWBlock) + 2 * tid;
            dst[0] = r[0];
            dst[1] = r[1];
        };
        // path p0 from the spinor stage sc and the link stage lc, while the weights and link
        // of path p0 + 1 and the spinors of path p0 + 2 are loaded; the wave writes and then
        // reads only its own rows of the tile, so a wave-level sync orders them. Every lane
        // issues the loads, the lanes of padded sites too (their site index is below the
        // padded row length and their neighbours are those of site 0, so the loads stay in
        // bounds; the data are not used): with the same loads in flight on every path
        // through the code, the compiler waits for exactly the loads an instruction needs
        auto path = [&](int p0, const SpStage& sc, SpStage& sn2, const LkStage& lc, LkStage& ln) {
            u32x4 wn[2];
            if (p0 + 1 < kPaths) {
                load_w(p0 + 1, wn);
                fetch_lk(p0 + 1, ln);
            }
            if (p0 + 2 < kPaths) fetch_sp(p0 + 2, sn2);
            // the matrix cores' second operand for row tile (colour) c: this lane's site,
            // channel cg (T0) or cg + 4 (T1), the four spins' (re, im) as bf16 -- exactly
            // the 8 consecutive columns of its row that a lane supplies in the product
            bf16x8 T0[3], T1[3];
            if (!real) {
                for (int c = 0; c < 3; ++c) T0[c] = T1[c] = bf16x8{};
            } else if (p0 == 0) {
                nn_rows_raw(sc.s0, T0);
                nn_rows_raw(sc.s1, T1);
            } else {
                const bool fwd = ((p0 - 1) & 1) == 0;
                cx<float> w[12], m[9];
                LinkBF lb;
                nn_link_matrix(lc.u, lc.d, lc.sg, m);
                nn_link_bf16(fwd, m, lb);
                nn_transport_dot2(lb, sc.s0, w);
                nn_rows(w, T0);
                nn_transport_dot2(lb, sc.s1, w);
                nn_rows(w, T1);
            }
            wb = wbuf + (p0 & 1) * (kWBlock / 2);
            // K = 64 per path in two steps of gfx950's doubled-K bf16 product (16 x 16 x 32),
            // channels 0..3 then 4..7; each lane reads 8 consecutive k of its column of the
            // path's weight block ([k/8][n][k%8] in LDS)
            for (int h = 0; h < 2; ++h) {
                const int kl = 32 * h + 8 * (lane >> 4);
                bf16x8 bf[NT];
                for (int j = 0; j < NT; ++j)
                    bf[j] = *(const bf16x8*)&wb[((kl >> 3) * 64 + j * 16 + (lane & 15)) * 8];
                for (int r = 0; r < 3; ++r)
                    for (int j = 0; j < NT; ++j)
                        acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[j], h ? T1[r] : T0[r],
                                                                           acc[r][j], 0, 0, 0);
            }
            if (p0 + 1 < kPaths) {
                // the next block into the other buffer (last read by every wave before the
                // previous barrier); the barrier also keeps every wave's reads of this path's
                // block ahead of its rewrite at the end of the next path
                store_w(p0 + 1, wn);
                __syncthreads();
            }
        };
        SpStage S0, S1, S2;
        LkStage LA, LB;  // path 0 has no link: LA first holds path 2's
        {
            u32x4 w0[2];
            load_w(0, w0);
            fetch_sp(0, S0);
            fetch_sp(1, S1);
            store_w(0, w0);
        }
        __syncthreads();
        // unrolled, so that the stage of each path is fixed at compile time; the last
        // two paths issue fewer loads
#pragma unroll
        for (int p0 = 0; p0 < kPaths; ++p0) {
            const int r3 = p0 % 3;
            if (p0 & 1) {
                if (r3 == 0) path(p0, S0, S2, LB, LA);
                else if (r3 == 1) path(p0, S1, S0, LB, LA);
                else path(p0, S2, S1, LB, LA);
            } else {
                if (r3 == 0) path(p0, S0, S2, LA, LB);
                else if (r3 == 1) path(p0, S1, S0, LA, LB);
                else path(p0, S2, S1, LA, LB);
            }
        }
    } else {
        // paths wave, wave + 4, wave + 8 of the single channel, one batch
        for (int p = wave; p < kPaths; p += 4) {
            cx<float> w[12];
            if (!real) {
                nn_put_rows<LS>(tile, sl, p * 8, zero12);
                continue;
            }
            if (p == 0) {
                load_spinor<PIN>(in[0], g.Vh, par, i, w);
            } else {
                int j;
                float sg;
                cx<float> u[6], d, sp[12];
                nn_path_setup(g, par, i, x, lex, p, links, dets, j, sg, u, d);
                load_spinor<PIN>(in[0], g.Vh, 1 - par, j, sp);
                cx<float> m[9];
                nn_link_matrix(u, d, sg, m);
                nn_apply_m(((p - 1) & 1) == 0, m, sp, w);
            }
            nn_put_rows<LS>(tile, sl, p * 8, w);
        }
        // zero padding columns 72..79
        for (int rr = threadIdx.x; rr < 192; rr += 256)
            *(uint4*)&tile[rr * LS + kPaths * 8] = uint4{0u, 0u, 0u, 0u};
        __syncthreads();  // the waves filled each other's rows
        mix_tile();
    }
    __syncthreads();  // the output block below reuses the tile
    if constexpr (MIXOUT) {
        // m_p = the layer's outputs rounded to bf16 (as the stored hidden channels would be)
        // times Bm, K = 64 in four steps of 16: step j takes the lane's acc[r][j] as its
        // operand, again as the transposed product (Bm^T first), so am[r][jm] holds row
        // 16 r + l % 16 and columns 16 jm + 4 (l / 16) + e of m, column (p * 4 + s) * 2 + re/im
        constexpr int NM = 5;  // 80 columns: 9 paths x 4 spins x re/im (72), padded
        f4 am[3][NM];
        for (int r = 0; r < 3; ++r)
            for (int jm = 0; jm < NM; ++jm) am[r][jm] = f4{0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < NT; ++j) {
            const int kl = j * 16 + 4 * (lane >> 4);
            s4 bf[NM];
            for (int jm = 0; jm < NM; ++jm)
                bf[jm] = *(const s4*)(Bm + (jm * 16 + (lane & 15)) * 64 + kl);
            for (int r = 0; r < 3; ++r) {
                const uint32_t h2[2] = {pack_bf16x2(acc[r][j][0], acc[r][j][1]),
                                        pack_bf16x2(acc[r][j][2], acc[r][j][3])};
                s4 a;
                __builtin_memcpy(&a, h2, 8);
                for (int jm = 0; jm < NM; ++jm)
                    am[r][jm] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf[jm], a, am[r][jm], 0, 0, 0);
            }
        }
        // staged as [path][chunk][site][8] like the outputs below, (re, im) pairs as one word
        uint16_t* ob = (uint16_t*)lds;
        for (int r = 0; r < 3; ++r)
            for (int jm = 0; jm < NM; ++jm)
                for (int h = 0; h < 2; ++h) {
                    int ms, c;
                    row_site(r, lane & 15, ms, c);
                    const int n = jm * 16 + 4 * (lane >> 4) + 2 * h;
                    if (n >= 72) continue;
                    const int p = n >> 3, sp = (n >> 1) & 3;
                    const int k = (sp * 3 + c) * 2;
                    *(uint32_t*)&ob[(p * 3 + (k >> 3)) * OROW + ms * 8 + (k & 7)] =
                        pack_bf16x2(am[r][jm][2 * h], am[r][jm][2 * h + 1]);
                }
        __syncthreads();
        const int mpar = (int)(q0 / Vp), mi0 = (int)(q0 - (long)mpar * Vp);
        for (int u = threadIdx.x; u < kPaths * 3 * 64; u += 256) {
            const int p = u / 192, rem = u - p * 192, ch = rem >> 6, site = rem & 63;
            if (mi0 + site >= g.Vh) continue;
            const uint4 raw = *(const uint4*)&ob[(p * 3 + ch) * OROW + site * 8];
            ((uint4*)out[p])[chunk_at(g.Vh, 3, mpar, ch, mi0 + site)] = raw;
        }
        return;
    }
    // outputs: row m = 3 * site + c, column n = (a * 4 + s) * 2 + re/im, rounded to bf16
    // (the conversion instruction) and staged in LDS as [channel][chunk][site][8] (the 64
    // sites are one aligned block of one parity; rows padded as in the tile), then written
    // as 16-byte chunks
    uint16_t* ob = (uint16_t*)lds;
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < NT; ++j)
            for (int h = 0; h < 2; ++h) {
                int ms, c;
                row_site(r, lane & 15, ms, c);
                const int n = j * 16 + 4 * (lane >> 4) + 2 * h;
                const int a = n >> 3, sp = (n >> 1) & 3;
                if (a >= COUT) continue;
                const int k = (sp * 3 + c) * 2;  // real index of the pair within the spinor
                *(uint32_t*)&ob[(a * 3 + (k >> 3)) * OROW + ms * 8 + (k & 7)] =
                    pack_bf16x2(acc[r][j][2 * h], acc[r][j][2 * h + 1]);
            }
    __syncthreads();
    const int opar = (int)(q0 / Vp), oi0 = (int)(q0 - (long)opar * Vp);
    for (int u = threadIdx.x; u < COUT * 3 * 64; u += 256) {
        const int a = u / 192, rem = u - a * 192, ch = rem >> 6, site = rem & 63;
        if (oi0 + site >= g.Vh) continue;
        const uint4 raw = *(const uint4*)&ob[(a * 3 + ch) * OROW + site * 8];
        ((uint4*)out[a])[chunk_at(g.Vh, 3, opar, ch, oi0 + site)] = raw;
    }
}

// ------------------------------------------------------------------ last layer: mix, then transport
//
// With one output channel the order of the two linear maps of a layer pays to be swapped:
// W_p acts on spin and channel, T_p on colour and site, so
//     out(x) = sum_p sum_b W_p[0][b] (T_p in_b)(x) = sum_p (T_p m_p)(x),
//     m_p(y) = sum_b W_p[0][b] in_b(y).
// Pass 1 forms the nine m_p at every site on the matrix cores (rows (site, colour), K = 8
// channels x 4 spins x re/im, N = 9 paths x 4 spins x re/im), storing them in bf16; pass 2
// is a plain stencil over them. Each site then gathers 9 spinors instead of 72.

// Bm[n][k]: n = (p*4 + s)*2 + re/im (72, padded to 80), k = (b*4 + t)*2 + re/im (64)
__global__ void nn_embed_mix_kernel(const float* W, uint16_t* Bm)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 80 * 64) return;
    const int n = tid / 64, k = tid - n * 64;
    float v = 0.f;
    if (n < 72) {
        const int p = n >> 3, sro = n & 7;            // (s, re/im) of the output
        const int b = k >> 3, tri = k & 7;            // (t, re/im) of the input
        v = embed(W, 8, 1, (p * 8 + b) * 8 + tri, sro);
    }
    Bm[tid] = float_to_bf16(v);
}

__global__ __launch_bounds__(256) void nn_mix_paths_kernel(Geom g, const void* const* in,
                                                           const uint16_t* Bm, void* const* mix)
{
    constexpr int KB = 64, LS = tile_stride(KB), NT = 5;
    // output staging in bf16: one row per (path, 16-byte chunk) of 64 sites x 8 halves,
    // padded by one chunk so that consecutive rows start 4 banks apart
    constexpr int ROW = 64 * 8 + 8;
    constexpr int TILE_B = 192 * LS * 2, OUT_B = 9 * 3 * ROW * 2;
    __shared__ __attribute__((aligned(16))) char lds[TILE_B > OUT_B ? TILE_B : OUT_B];
    uint16_t* tile = (uint16_t*)lds;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Vp = padded(g.Vh);
    const long q0 = nn_block_q0(Vp);
    const int par = (int)(q0 / Vp), i0 = (int)(q0 - (long)par * Vp);
    const int i = i0 + lane;
    const cx<float> zero12[12] = {};
    // rows of the tile: the site's eight input channels (channels wave and wave + 4)
    if (i < g.Vh) {
        cx<float> w0[12], w1[12];
        load_spinor<BF16S>(in[wave], g.Vh, par, i, w0);
        load_spinor<BF16S>(in[wave + 4], g.Vh, par, i, w1);
        nn_put_rows<LS>(tile, lane, wave * 8, w0);
        nn_put_rows<LS>(tile, lane, (wave + 4) * 8, w1);
    } else {
        nn_put_rows<LS>(tile, lane, wave * 8, zero12);
        nn_put_rows<LS>(tile, lane, (wave + 4) * 8, zero12);
    }
    __syncthreads();
    f4 acc[3][NT];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < NT; ++j) acc[r][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < KB; kk += 16) {
        const int kl = kk + 4 * (lane >> 4);
        s4 bf[NT];
        for (int j = 0; j < NT; ++j)
            bf[j] = *(const s4*)(Bm + (j * 16 + (lane & 15)) * KB + kl);
        for (int r = 0; r < 3; ++r) {
            const s4 a = *(const s4*)&tile[(wave * 48 + r * 16 + (lane & 15)) * LS + kl];
            for (int j = 0; j < NT; ++j)
                acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bf[j], acc[r][j], 0, 0, 0);
        }
    }
    __syncthreads();
    // outputs rounded to bf16 (the conversion instruction, as for the other bf16 fields)
    // and staged as [path][chunk][site][8], then written as 16-byte chunks
    uint16_t* ob = (uint16_t*)lds;
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < NT; ++j)
            for (int e = 0; e < 4; ++e) {
                const int m = wave * 48 + r * 16 + 4 * (lane >> 4) + e;
                const int n = j * 16 + (lane & 15);
                if (n >= 72) continue;
                const int ms = m / 3, c = m - ms * 3;
                const int p = n >> 3, sp = (n >> 1) & 3, ri = n & 1;
                const int k = (sp * 3 + c) * 2 + ri;  // real index within the spinor
                ob[(p * 3 + (k >> 3)) * ROW + ms * 8 + (k & 7)] =
                    (uint16_t)(pack_bf16x2(acc[r][j][e], 0.f) & 0xFFFFu);
            }
    __syncthreads();
    for (int u = threadIdx.x; u < 9 * 3 * 64; u += 256) {
        const int p = u / 192, rem = u - p * 192, ch = rem >> 6, site = rem & 63;
        if (i0 + site >= g.Vh) continue;
        const uint4 raw = *(const uint4*)&ob[(p * 3 + ch) * ROW + site * 8];
        ((uint4*)mix[p])[chunk_at(g.Vh, 3, par, ch, i0 + site)] = raw;
    }
}

// out(x) = m_0(x) + sum_{p = 1..8} (T_p m_p)(x)   (FP32 output)
__global__ __launch_bounds__(256) void nn_transport_sum_kernel(Geom g, const void* const* mix,
                                                               float* out, const void* links,
                                                               const void* dets)
{
    // 256-site blocks of the two parities alternate, XCD-contiguously (as nn_block_q0)
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    const int par = w & 1;
    const int i = (w >> 1) * 256 + (int)threadIdx.x;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    cx<float> acc[12];
    load_spinor<BF16S>(mix[0], g.Vh, par, i, acc);
#pragma unroll 1
    for (int p = 1; p < kPaths; ++p) {
        int j;
        float sg;
        cx<float> u[6], d;
        nn_path_setup(g, par, i, x, lex, p, links, dets, j, sg, u, d);
        u32x4 raw[3];
        const long b0 = chunk_at(g.Vh, 3, 1 - par, 0, j);
#pragma unroll
        for (int k = 0; k < 3; ++k) raw[k] = ((const u32x4*)mix[p])[b0 + (long)k * kSB];
        cx<float> m[9];
        LinkBF lb;
        nn_link_matrix(u, d, sg, m);
        nn_link_bf16(((p - 1) & 1) == 0, m, lb);
        nn_transport_dot2<true>(lb, raw, acc);
    }
    store_spinor<F32>(out, g.Vh, par, i, acc);
}

__global__ void fill_kernel(uint32_t* p, long n)
{
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p[k] = 0u;
}

__global__ void adam_kernel(float* w, float* m, float* v, const float* g, int n, float lr,
                            float b1, float b2, float c1, float c2, float eps, float gscale)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gr = g[k] * gscale;
    m[k] = b1 * m[k] + (1.f - b1) * gr;
    v[k] = b2 * v[k] + (1.f - b2) * gr * gr;
    w[k] -= lr * (m[k] / c1) / (sqrtf(v[k] / c2) + eps);
}

// loss terms: d = out - e (stored in `d`), sum |d|^2
struct LossDiff {
    static constexpr int NS = 1;
    const void* out;
    const void* e;
    void* d;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        cx<float> o[4], t[4];
        ld4<F32, float>(out, Vh, u.par, u.g, u.i, o);
        ld4<F32, float>(e, Vh, u.par, u.g, u.i, t);
        for (int k = 0; k < 4; ++k) {
            o[k] = o[k] - t[k];
            acc[0] += (double)o[k].re * o[k].re + (double)o[k].im * o[k].im;
        }
        st4<F32, float>(d, Vh, u.par, u.g, u.i, o);
    }
};

// ------------------------------------------------------------------ host side

struct NnWork {
    float* act[kLayers + 1][8];  // channel fields per layer boundary (FP32 space; the hidden
                                 // ones hold bf16 fields in the bf16 forward pass)
    float* grad[2][8];           // gradient channel fields (ping-pong)
    float* efield;               // target (FP32)
    void* A;                     // transported rows, [Mpad][Kmax]
    float* dA;                   // [Mpad][Kmax] (training only)
    void* G;                     // [Mpad][Nmax]
    void* Bt;                    // [Nmax][Kmax]
    void* Bk;                    // [Kmax][Nmax]
    float* part;                 // [nsplit][Kmax][Nmax]
    float* dB;                   // [Kmax][Nmax]
    void* mix[kPaths];           // bf16 fields m_p of the last layer's path mixing
    uint16_t* Bm;                // [80][64] bf16: the last layer's mixing matrix
    uint16_t* Bl;                // [9][16][64][4] bf16: the 8-channel layer's weights as
                                 // the fused kernel's LDS image
    float** ptrs;                // device pointer tables (8 pointers per slot)
    char* end;
};

constexpr int kSplit = 64;

// need_A: the materialised transport matrix A (FP32-operand forward passes, training)
size_t nn_layout(const qdw_op* op, bool training, char* base, NnWork* W, bool need_A = true)
{
    const Geom& g = op->g;
    const size_t fb = spinor_bytes(g, F32);
    const long Mp = rows_padded(g);
    size_t off = 0;
    auto take = [&](size_t n) {
        char* at = base ? base + off : nullptr;
        off += (n + 255) & ~(size_t)255;
        return at;
    };
    for (int l = 0; l <= kLayers; ++l)
        for (int c = 0; c < 8; ++c) W->act[l][c] = c < kCh[l] ? (float*)take(fb) : nullptr;
    for (int h = 0; h < 2; ++h)
        for (int c = 0; c < 8; ++c) W->grad[h][c] = training ? (float*)take(fb) : nullptr;
    W->efield = training ? (float*)take(fb) : nullptr;
    W->A = need_A || training ? take((size_t)Mp * kMaxK * 4) : nullptr;
    for (int p = 0; p < kPaths; ++p) W->mix[p] = take(spinor_bytes(g, BF16S));
    W->Bm = (uint16_t*)take(80 * 64 * 2);
    W->Bl = (uint16_t*)take((size_t)kPaths * kWBlock);
    W->dA = training ? (float*)take((size_t)Mp * kMaxK * 4) : nullptr;
    W->G = training ? take((size_t)Mp * kMaxN * 4) : nullptr;
    W->Bt = take((size_t)kMaxN * kMaxK * 4);
    W->Bk = take((size_t)kMaxN * kMaxK * 4);
    W->part = training ? (float*)take((size_t)kSplit * kMaxN * kMaxK * 4) : nullptr;
    W->dB = training ? (float*)take((size_t)kMaxN * kMaxK * 4) : nullptr;
    W->ptrs = (float**)take(64 * sizeof(float*));
    return off + 256;
}

int set_ptrs(float** dev, float* const* host, int n, int slot, hipStream_t st)
{
    QDW_HIP(hipMemcpyAsync(dev + 8 * slot, host, sizeof(float*) * n, hipMemcpyHostToDevice, st));
    return QDW_OK;
}

int zero_dev(void* p, size_t bytes, hipStream_t st)
{
    const long n = (long)(bytes / 4);
    fill_kernel<<<1024, 256, 0, st>>>((uint32_t*)p, n);
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

// forward through all layers, input already in act[0][0]; keeps every layer's input
// (keep_hidden, needed by the gradients), or, in bf16 inference passes without it, fuses
// the last layer's path mixing into the 8 -> 8 layer so that the second hidden layer's
// channels never go to memory
template <bool F32M>
int forward(qdw_op* op, const float* weights, NnWork& W, hipStream_t st, bool keep_hidden = true)
{
    const Geom& g = op->g;
    const long Mp = rows_padded(g);
    const long nq = 2L * padded(g.Vh);
    int rc;
    for (int l = 0; l < kLayers; ++l) {
        const int Cin = kCh[l], Cout = kCh[l + 1], Kp = layer_K(l), Np = layer_N(l);
        if ((rc = set_ptrs(W.ptrs, W.act[l], Cin, 0, st))) return rc;
        if ((rc = set_ptrs(W.ptrs, W.act[l + 1], Cout, 1, st))) return rc;
        nn_embed_kernel<F32M><<<(Kp * Np + 255) / 256, 256, 0, st>>>(
            weights + 2 * layer_w_offset(l), Cin, Cout, Kp, Np, W.Bt, W.Bk);
        QDW_LAUNCH_CHECK();
        if constexpr (!F32M) {
            // hidden activations (between the layers) are stored in bf16, the network's
            // input and output in FP32
            const unsigned nb = (unsigned)(nq / 64);
            const void* L = op->links[F32];
            const void* D = op->det[F32];
            const void* const* pin = (const void* const*)W.ptrs;
            void* const* pout = (void* const*)(W.ptrs + 8);
            if (Cin == 1) {
                nn_layer_fused_kernel<1, 8, F32, BF16S><<<nb, 256, 0, st>>>(g, Kp, pin, W.Bt, nullptr,
                                                                             pout, L, D);
                QDW_LAUNCH_CHECK();
            } else if (Cout == 8) {
                nn_embed_lds_kernel<<<(kPaths * 64 * 64 + 255) / 256, 256, 0, st>>>(
                    (const uint16_t*)W.Bt, Kp, W.Bl);
                QDW_LAUNCH_CHECK();
                if (keep_hidden) {
                    nn_layer_fused_kernel<8, 8, BF16S, BF16S><<<nb, 256, 0, st>>>(
                        g, Kp, pin, W.Bt, W.Bl, pout, L, D);
                } else {
                    // the last layer's mixing matrix first: its product runs in this launch
                    if ((rc = set_ptrs(W.ptrs, (float* const*)W.mix, kPaths, 3, st))) return rc;
                    nn_embed_mix_kernel<<<(80 * 64 + 255) / 256, 256, 0, st>>>(
                        weights + 2 * layer_w_offset(l + 1), W.Bm);
                    QDW_LAUNCH_CHECK();
                    nn_layer_fused_kernel<8, 8, BF16S, BF16S, true><<<nb, 256, 0, st>>>(
                        g, Kp, pin, W.Bt, W.Bl, (void* const*)(W.ptrs + 24), L, D, W.Bm);
                }
                QDW_LAUNCH_CHECK();
            } else {
                // one output channel: mix the paths first (already done by the 8 -> 8
                // layer's launch when the hidden channels are not kept), then transport 9
                // fields
                if (keep_hidden) {
                    if ((rc = set_ptrs(W.ptrs, (float* const*)W.mix, kPaths, 3, st))) return rc;
                    nn_embed_mix_kernel<<<(80 * 64 + 255) / 256, 256, 0, st>>>(
                        weights + 2 * layer_w_offset(l), W.Bm);
                    QDW_LAUNCH_CHECK();
                    nn_mix_paths_kernel<<<nb, 256, 0, st>>>(g, pin, W.Bm,
                                                            (void* const*)(W.ptrs + 24));
                    QDW_LAUNCH_CHECK();
                }
                nn_transport_sum_kernel<<<2 * ((g.Vh + 255) / 256), 256, 0, st>>>(
                    g, (const void* const*)(W.ptrs + 24), W.act[l + 1][0], L, D);
                QDW_LAUNCH_CHECK();
            }
        } else {
            nn_transport_kernel<F32M, F32><<<(unsigned)((nq * Cin + 255) / 256), 256, 0, st>>>(
                g, Cin, Kp, Mp, (const void* const*)W.ptrs, W.A, op->links[F32], op->det[F32]);
            QDW_LAUNCH_CHECK();
            nn_gemm_out_kernel<F32M><<<(unsigned)(Mp / 64), 256, 0, st>>>(g, Kp, Np, Cout, Mp, W.A,
                                                                          W.Bt, W.ptrs + 8);
            QDW_LAUNCH_CHECK();
        }
    }
    return QDW_OK;
}

// backward from the real gradient of the network output (grad[0][0], times gscale);
// accumulates dL/dRe W + i dL/dIm W into dW and leaves the input gradient in grad[x][0]
template <bool F32M>
int backward(qdw_op* op, const float* weights, float* dW, NnWork& W, float gscale, hipStream_t st,
             float** gin_out)
{
    const Geom& g = op->g;
    const long Mp = rows_padded(g);
    const long nq = 2L * padded(g.Vh);
    const long M = rows_of(g);
    int rc;
    int cur = 0;  // grad[cur] holds the gradient of layer l's output
    for (int l = kLayers - 1; l >= 0; --l) {
        const int Cin = kCh[l], Cout = kCh[l + 1], Kp = layer_K(l), Np = layer_N(l);
        // recompute this layer's transported input rows (hidden activations are bf16 in
        // the bf16 forward pass)
        if ((rc = set_ptrs(W.ptrs, W.act[l], Cin, 0, st))) return rc;
        const unsigned ntb = (unsigned)((nq * Cin + 255) / 256);
        if (F32M || l == 0)
            nn_transport_kernel<F32M, F32><<<ntb, 256, 0, st>>>(
                g, Cin, Kp, Mp, (const void* const*)W.ptrs, W.A, op->links[F32], op->det[F32]);
        else
            nn_transport_kernel<F32M, BF16S><<<ntb, 256, 0, st>>>(
                g, Cin, Kp, Mp, (const void* const*)W.ptrs, W.A, op->links[F32], op->det[F32]);
        QDW_LAUNCH_CHECK();
        nn_embed_kernel<F32M><<<(Kp * Np + 255) / 256, 256, 0, st>>>(
            weights + 2 * layer_w_offset(l), Cin, Cout, Kp, Np, W.Bt, W.Bk);
        QDW_LAUNCH_CHECK();
        // G rows from the output gradient
        if ((rc = set_ptrs(W.ptrs, W.grad[cur], Cout, 1, st))) return rc;
        nn_pack_g_kernel<F32M><<<(unsigned)((nq + 255) / 256), 256, 0, st>>>(
            g, Cout, Np, W.ptrs + 8, l == kLayers - 1 ? gscale : 1.f, W.G);
        QDW_LAUNCH_CHECK();
        // weight gradient dB = A^T G
        const long rows_per = ((M + kSplit - 1) / kSplit + 15) & ~15L;
        nn_gemm_db_kernel<F32M><<<dim3(Kp / 16, kSplit), 256, 0, st>>>(M, Kp, Np, (int)rows_per,
                                                                      Mp, W.A, W.G, W.part);
        QDW_LAUNCH_CHECK();
        nn_reduce_db_kernel<<<(Kp * Np + 255) / 256, 256, 0, st>>>(W.part, kSplit, Kp * Np, W.dB);
        QDW_LAUNCH_CHECK();
        const int nw = kPaths * Cout * Cin * 16;
        nn_dw_kernel<<<(nw + 255) / 256, 256, 0, st>>>(W.dB, Cin, Cout, Np,
                                                       dW + 2 * layer_w_offset(l));
        QDW_LAUNCH_CHECK();
        // input gradient dA = G B^T, then the adjoint transport
        nn_gemm_da_kernel<F32M><<<(unsigned)(Mp / 64), 256, 0, st>>>(Kp, Np, Mp, W.G, W.Bk, W.dA);
        QDW_LAUNCH_CHECK();
        if ((rc = set_ptrs(W.ptrs, W.grad[1 - cur], Cin, 2, st))) return rc;
        nn_transport_adj_kernel<<<(unsigned)((nq * Cin + 255) / 256), 256, 0, st>>>(
            g, Cin, Mp, W.dA, W.ptrs + 16, op->links[F32], op->det[F32]);
        QDW_LAUNCH_CHECK();
        cur = 1 - cur;
    }
    if (gin_out) *gin_out = W.grad[cur][0];
    return QDW_OK;
}

char* align_work(void* work) { return (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255); }

}  // namespace

size_t nn_precond_workspace(const qdw_op* op)
{
    NnWork W;
    return nn_layout(op, false, nullptr, &W, false);  // bf16 forward only: no A
}

// phi = N(rho): rho, phi FP64 eo-SoA fields; |rho| given (sets the FP32 scale)
int nn_precondition(qdw_op* op, const void* weights, const void* rho, void* phi, double rho_norm,
                    char* work, hipStream_t st)
{
    NnWork W;
    nn_layout(op, false, work, &W, false);
    const Geom& g = op->g;
    int rc;
    if (!(rho_norm > 0.0)) return run_map(op, Zero<F64>{phi, g.Vh}, st);
    const double s = std::sqrt(24.0 * g.V) / rho_norm;
    if ((rc = run_map(op, ScaleNorm<F64, F32>{rho, W.act[0][0], s, g.Vh}, st,
                      op->scalars + S_TMP + 2)))
        return rc;
    if ((rc = forward<false>(op, (const float*)weights, W, st, false))) return rc;
    return run_map(op, Axpby<F32, F64>{W.act[kLayers][0], phi, 1.0 / s, 0.0, g.Vh}, st);
}

}  // namespace qdw

using namespace qdw;

extern "C" int qdw_nn_weight_count(void) { return total_weights(); }

extern "C" size_t qdw_nn_workspace_bytes(const qdw_op* op, int training)
{
    if (!op) return 0;
    NnWork W;
    return nn_layout(op, training != 0, nullptr, &W);
}

extern "C" int nn_forward(qdw_op* op, const float* weights, const void* in, void* out, int f32_mixing,
                          void* work, size_t work_bytes, void* stream)
{
    QDW_CHECK(op && weights && in && out && work, QDW_EINVAL, "nn_forward: null argument");
    QDW_CHECK(work_bytes >= qdw_nn_workspace_bytes(op, 0), QDW_EWORKSPACE,
              "nn_forward: workspace smaller than qdw_nn_workspace_bytes(op, 0)");
    hipStream_t st = (hipStream_t)stream;
    NnWork W;
    nn_layout(op, false, align_work(work), &W);
    const Geom& g = op->g;
    int rc;
    if ((rc = run_map(op, Axpby<F64, F32>{in, W.act[0][0], 1.0, 0.0, g.Vh}, st))) return rc;
    rc = f32_mixing ? forward<true>(op, weights, W, st) : forward<false>(op, weights, W, st, false);
    if (rc) return rc;
    return run_map(op, Axpby<F32, F64>{W.act[kLayers][0], out, 1.0, 0.0, g.Vh}, st);
}

extern "C" int nn_backward(qdw_op* op, const float* weights, const void* in, const void* gout,
                           float* dW, void* gin, int f32_mixing, void* work, size_t work_bytes,
                           void* stream)
{
    QDW_CHECK(op && weights && in && gout && dW && gin && work, QDW_EINVAL,
              "nn_backward: null argument");
    QDW_CHECK(work_bytes >= qdw_nn_workspace_bytes(op, 1), QDW_EWORKSPACE,
              "nn_backward: workspace smaller than qdw_nn_workspace_bytes(op, 1)");
    hipStream_t st = (hipStream_t)stream;
    NnWork W;
    nn_layout(op, true, align_work(work), &W);
    const Geom& g = op->g;
    int rc;
    if ((rc = zero_dev(dW, sizeof(float) * 2 * total_weights(), st))) return rc;
    if ((rc = run_map(op, Axpby<F64, F32>{in, W.act[0][0], 1.0, 0.0, g.Vh}, st))) return rc;
    rc = f32_mixing ? forward<true>(op, weights, W, st) : forward<false>(op, weights, W, st);
    if (rc) return rc;
    if ((rc = run_map(op, Axpby<F64, F32>{gout, W.grad[0][0], 1.0, 0.0, g.Vh}, st))) return rc;
    float* gi = nullptr;
    rc = f32_mixing ? backward<true>(op, weights, dW, W, 1.f, st, &gi)
                    : backward<false>(op, weights, dW, W, 1.f, st, &gi);
    if (rc) return rc;
    return run_map(op, Axpby<F32, F64>{gi, gin, 1.0, 0.0, g.Vh}, st);
}

namespace {

// x (pair storage precision P) -> FP32 field times s; |x|^2 of the input when want_norm
template <int P>
int pair_to_f32(qdw_op* op, const void* x, float* y, double s, hipStream_t st)
{
    return run_map(op, Axpby<P, F32>{x, y, s, 0.0, op->g.Vh}, st);
}

int pair_norm2(qdw_op* op, const void* x, int prec, double* out, hipStream_t st)
{
    int rc;
    switch (prec) {
    case F64: rc = run_map(op, Norm2<F64>{x, op->g.Vh}, st, op->scalars + S_TMP); break;
    case F32: rc = run_map(op, Norm2<F32>{x, op->g.Vh}, st, op->scalars + S_TMP); break;
    default: rc = run_map(op, Norm2<BF16S>{x, op->g.Vh}, st, op->scalars + S_TMP); break;
    }
    if (rc) return rc;
    return read_scalars(op, S_TMP, 1, out, st);
}

int pair_convert(qdw_op* op, const void* x, int prec, float* y, double s, hipStream_t st)
{
    switch (prec) {
    case F64: return pair_to_f32<F64>(op, x, y, s, st);
    case F32: return pair_to_f32<F32>(op, x, y, s, st);
    default: return pair_to_f32<BF16S>(op, x, y, s, st);
    }
}

}  // namespace

extern "C" int nn_train_step(qdw_op* op, float* weights, float* adam, int step, double lr,
                             const void* const* rho, const void* const* err, int nbatch,
                             qdw_prec pair_prec, int loss_kind, double* loss, void* work,
                             size_t work_bytes, void* stream)
{
    QDW_CHECK(loss_kind == 0 || loss_kind == 1, QDW_EINVAL, "nn_train_step: loss_kind 0 or 1");
    QDW_CHECK(op && weights && adam && rho && err && loss && work && nbatch >= 1 && step >= 1,
              QDW_EINVAL, "nn_train_step: bad argument");
    QDW_CHECK(pair_prec == QDW_F64 || pair_prec == QDW_F32 || pair_prec == QDW_BF16S, QDW_EINVAL,
              "nn_train_step: pairs must be QDW_F64, QDW_F32 or QDW_BF16S fields");
    QDW_CHECK(work_bytes >= qdw_nn_workspace_bytes(op, 1) + sizeof(float) * 2 * total_weights() + 512,
              QDW_EWORKSPACE, "nn_train_step: workspace smaller than "
                              "qdw_nn_workspace_bytes(op, 1) + 8 * qdw_nn_weight_count() + 512");
    hipStream_t st = (hipStream_t)stream;
    NnWork W;
    char* base = align_work(work);
    const size_t nb = nn_layout(op, true, base, &W);
    float* dW = (float*)(base + ((nb + 255) & ~(size_t)255));
    const int nw2 = 2 * total_weights();
    const Geom& g = op->g;
    int rc;
    if ((rc = zero_dev(dW, sizeof(float) * nw2, st))) return rc;
    double total = 0.0;
    for (int k = 0; k < nbatch; ++k) {
        // scale the pair so that the residual has unit component size (the map is linear)
        double r2;
        if ((rc = pair_norm2(op, rho[k], pair_prec, &r2, st))) return rc;
        QDW_CHECK(r2 > 0.0, QDW_EINVAL, "nn_train_step: a residual is zero");
        const double s = std::sqrt(24.0 * g.V / r2);
        if ((rc = pair_convert(op, rho[k], pair_prec, W.act[0][0], s, st))) return rc;
        if ((rc = pair_convert(op, err[k], pair_prec, W.efield, s, st))) return rc;
        double e2;
        if ((rc = run_map(op, Norm2<F32>{W.efield, g.Vh}, st, op->scalars + S_TMP))) return rc;
        if ((rc = read_scalars(op, S_TMP, 1, &e2, st))) return rc;
        if ((rc = forward<false>(op, weights, W, st))) return rc;
        double d2;
        if ((rc = run_map(op, LossDiff{W.act[kLayers][0], W.efield, W.grad[0][0], g.Vh}, st,
                          op->scalars + S_TMP)))
            return rc;
        if ((rc = read_scalars(op, S_TMP, 1, &d2, st))) return rc;
        double denom = e2;
        if (loss_kind == 1) {
            // D-norm: d = N(rho) - e  ->  t = D d, |t|^2, gradient direction D^+ t; the
            // normalisation |D e|^2 is |rho|^2 of the stored pair
            float* t = W.grad[1][0];
            float* De = W.grad[1][1];
            if ((rc = dw_launch(op, W.grad[0][0], t, F32, false, st))) return rc;
            if ((rc = run_map(op, Norm2<F32>{t, g.Vh}, st, op->scalars + S_TMP))) return rc;
            if ((rc = read_scalars(op, S_TMP, 1, &d2, st))) return rc;
            if ((rc = dw_launch(op, W.efield, De, F32, false, st))) return rc;
            if ((rc = run_map(op, Norm2<F32>{De, g.Vh}, st, op->scalars + S_TMP))) return rc;
            if ((rc = read_scalars(op, S_TMP, 1, &denom, st))) return rc;
            if ((rc = dw_launch(op, t, W.grad[0][0], F32, true, st))) return rc;
        }
        total += d2 / denom;
        // dL/d(out re, im) = 2 (out - e) / |e|^2, or 2 D^+ D (out - e) / |D e|^2, batch mean
        const float gs = (float)(2.0 / (denom * nbatch));
        if ((rc = backward<false>(op, weights, dW, W, gs, st, nullptr))) return rc;
    }
    *loss = total / nbatch;
    const float b1 = 0.9f, b2 = 0.999f;
    adam_kernel<<<(nw2 + 255) / 256, 256, 0, st>>>(weights, adam, adam + nw2, dW, nw2, (float)lr, b1,
                                                   b2, 1.f - std::pow(b1, (float)step),
                                                   1.f - std::pow(b2, (float)step), 1e-8f, 1.f);
    QDW_LAUNCH_CHECK();
    QDW_HIP(hipStreamSynchronize(st));
    return QDW_OK;
}
