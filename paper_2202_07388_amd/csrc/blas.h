// blas.h -- fused BLAS-1 on eo-SoA spinor fields with FP64 reductions.
//
// The paper (Sec. 2.1) keeps every reduction variable in binary64 whatever the working
// type of the vectors; here every lane accumulates its products in FP64 and the partial
// sums are combined across the wavefront (shuffles), the workgroup (LDS) and the grid
// (a second single-workgroup pass) in a fixed order, so results are bitwise
// reproducible run to run.
//
// Unit of work: 4 complex numbers of one site, (parity, group g in 0..2, site i). Fields
// of different storage precisions are addressed by the same unit, so mixed-precision
// kernels (FP32 solution, FP16 residual) pair the same lattice components.
#pragma once

#include "qdw_host.h"

namespace qdw {

// ---------------------------------------------------------------- unit load / store

template <int P, typename R>
__device__ __forceinline__ void ld4(const void* f, int Vh, int par, int g, int i, cx<R> v[4])
{
    using T = Traits<P>;
    constexpr int CPC = T::PER_CHUNK / 2;        // complex per chunk
    constexpr int NCH = 4 / CPC;                 // chunks per unit
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        Chunk<P> c = load_chunk_cached<P>(f, chunk_at(Vh, T::SPIN_CHUNKS, par, g * NCH + k, i));
#pragma unroll
        for (int j = 0; j < CPC; ++j)
            v[k * CPC + j] = {(R)to_real<P>(c.v[2 * j]), (R)to_real<P>(c.v[2 * j + 1])};
    }
}

template <int P, typename R>
__device__ __forceinline__ void st4(void* f, int Vh, int par, int g, int i, const cx<R> v[4])
{
    using T = Traits<P>;
    using RT = typename T::real;
    constexpr int CPC = T::PER_CHUNK / 2;
    constexpr int NCH = 4 / CPC;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
        Chunk<P> c;
#pragma unroll
        for (int j = 0; j < CPC; ++j) {
            c.v[2 * j] = to_store<P>((RT)v[k * CPC + j].re);
            c.v[2 * j + 1] = to_store<P>((RT)v[k * CPC + j].im);
        }
        const long at = chunk_at(Vh, T::SPIN_CHUNKS, par, g * NCH + k, i);
        uint4 raw;
        __builtin_memcpy(&raw, &c, 16);
        ((uint4*)f)[at] = raw;
    }
}

struct Unit { int par, g, i; };

__device__ __forceinline__ Unit unit_of(long u, int Vh)
{
    const long per = 3L * Vh;
    Unit r;
    r.par = (int)(u / per);
    const long rem = u - (long)r.par * per;
    r.g = (int)(rem / Vh);
    r.i = (int)(rem - (long)r.g * Vh);
    return r;
}

// ---------------------------------------------------------------- reductions

template <int NS>
__device__ __forceinline__ void block_reduce_store(double acc[NS], double* partial)
{
    __shared__ double red[4][NS > 0 ? NS : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        const int k = threadIdx.x;
        partial[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// grid-stride map over units; F::NS doubles reduced per workgroup into partials
template <class F>
__global__ __launch_bounds__(256) void map_kernel(long nunits, int Vh, F f, double* partials)
{
    double acc[F::NS > 0 ? F::NS : 1];
#pragma unroll
    for (int k = 0; k < (F::NS > 0 ? F::NS : 1); ++k) acc[k] = 0.0;
    for (long u = (long)blockIdx.x * blockDim.x + threadIdx.x; u < nunits;
         u += (long)gridDim.x * blockDim.x) {
        const Unit w = unit_of(u, Vh);
        f(w, acc);
    }
    if constexpr (F::NS > 0) block_reduce_store<F::NS>(acc, partials + (long)blockIdx.x * F::NS);
}

// scalar programs run by the finalising workgroup after the sums are formed
enum FinOp {
    FIN_STORE = 0,   // out[j] = sum_j
    FIN_CG_ALPHA,    // out = CG scalars: pap = sum_0; alpha = rr / pap
    FIN_CG_BETA,     // out = CG scalars: rrnew = sum_0; beta = rrnew / rr; rr = rrnew
    FIN_GCR_NORM,    // out = GCR scalars, step k: b_k = sqrt(sum_0), c_k = (sum_1 + i sum_2)/b_k,
                     //   coefficients 1/b_k and c_k/b_k for the update pass
};

// GCR scalar block (doubles): a[k][l] complex at 2*(16*k + l), b_k at G_B + k,
// c_k complex at G_C + 2k, update coefficients at G_COEF (1/b, Re c/b, Im c/b)
constexpr int kMaxKv = 16;
enum { G_A = 0, G_B = 2 * kMaxKv * kMaxKv, G_C = G_B + kMaxKv, G_COEF = G_C + 2 * kMaxKv,
       G_NORM = G_COEF + 4, G_SIZE = G_NORM + 4 };

// scalar slots of the CG solver
enum { S_RR = 0, S_PAP = 1, S_ALPHA = 2, S_RRNEW = 3, S_BETA = 4, S_TMP = 8 };

// Body of the finalising pass (one workgroup of 256 lanes): sums the per-workgroup
// partials in a fixed order (strided per lane, then a fixed tree), then runs the scalar
// program `op`.
__device__ inline void finalize_body(const double* partials, int nblk, int ns, double* out,
                                     int op, int k)
{
    __shared__ double red[256];
    __shared__ double sums[kMaxScalars];
    for (int j = 0; j < ns; ++j) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) s += partials[(long)b * ns + j];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) sums[j] = red[0];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    switch (op) {
    case FIN_STORE:
        for (int j = 0; j < ns; ++j) out[j] = sums[j];
        break;
    case FIN_CG_ALPHA:  // a vanishing direction leaves the iterate unchanged
        out[S_PAP] = sums[0];
        out[S_ALPHA] = sums[0] != 0.0 ? out[S_RR] / sums[0] : 0.0;
        break;
    case FIN_CG_BETA:
        out[S_RRNEW] = sums[0];
        out[S_BETA] = out[S_RR] != 0.0 ? sums[0] / out[S_RR] : 0.0;
        out[S_RR] = sums[0];
        break;
    case FIN_GCR_NORM: {
        const double b = sqrt(sums[0]);
        const double ib = b > 0.0 ? 1.0 / b : 0.0;
        out[G_B + k] = b;
        out[G_C + 2 * k] = sums[1] * ib;
        out[G_C + 2 * k + 1] = sums[2] * ib;
        out[G_COEF] = ib;
        out[G_COEF + 1] = sums[1] * ib * ib;
        out[G_COEF + 2] = sums[2] * ib * ib;
        break;
    }
    default:
        break;
    }
}

__global__ void finalize_kernel(const double* partials, int nblk, int ns, double* out, int op,
                                int k);

struct Reducer {
    int nblk;   // workgroups of the map launch (fixed per field size: deterministic)
};

inline int map_blocks(long nunits)
{
    long b = (nunits + 256 * 8 - 1) / (256 * 8);
    if (b > kMaxPartials) b = kMaxPartials;
    if (b < 1) b = 1;
    return (int)b;
}

// launch F over all 3V units of op's lattice, or over the first nu units when nu > 0
// (3 Vh: the even half), and (if F::NS > 0) finalise into scalars
template <class F>
int run_map(const qdw_op* op, const F& f, hipStream_t st, double* out = nullptr,
            int fin = FIN_STORE, int k = 0, long nu = 0)
{
    const long nunits = nu > 0 ? nu : 3L * op->g.V;
    const int nb = map_blocks(nunits);
    map_kernel<F><<<nb, 256, 0, st>>>(nunits, op->g.Vh, f, op->partials);
    QDW_LAUNCH_CHECK();
    if constexpr (F::NS > 0) {
        finalize_kernel<<<1, 256, 0, st>>>(op->partials, nb, F::NS, out ? out : op->scalars,
                                           fin, k);
        QDW_LAUNCH_CHECK();
    }
    return QDW_OK;
}

// ---------------------------------------------------------------- functors

template <int P>
struct Norm2 {
    static constexpr int NS = 1;
    const void* x;
    int Vh;
    __device__ void operator()(const Unit& w, double* acc) const
    {
        cx<double> v[4];
        ld4<P, double>(x, Vh, w.par, w.g, w.i, v);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[0] += v[k].re * v[k].re + v[k].im * v[k].im;
    }
};

// y = a x + b y, a and b real host scalars (no reduction)
template <int PX, int PY>
struct Axpby {
    static constexpr int NS = 0;
    const void* x;
    void* y;
    double a, b;
    int Vh;
    __device__ void operator()(const Unit& w, double*) const
    {
        using R = typename Traits<(PX == F64 && PY == F64) ? F64 : F32>::real;
        cx<R> vx[4], vy[4];
        ld4<PX, R>(x, Vh, w.par, w.g, w.i, vx);
        if (b != 0.0) ld4<PY, R>(y, Vh, w.par, w.g, w.i, vy);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cx<R> t = scale(vx[k], (R)a);
            if (b != 0.0) t = t + scale(vy[k], (R)b);
            vy[k] = t;
        }
        st4<PY, R>(y, Vh, w.par, w.g, w.i, vy);
    }
};

// y = s x (down-conversion with scaling) and |y|^2 of the stored values
template <int PX, int PY>
struct ScaleNorm {
    static constexpr int NS = 1;
    const void* x;
    void* y;
    double s;
    int Vh;
    __device__ void operator()(const Unit& w, double* acc) const
    {
        cx<double> vx[4];
        ld4<PX, double>(x, Vh, w.par, w.g, w.i, vx);
        cx<double> vy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) vy[k] = scale(vx[k], s);
        st4<PY, double>(y, Vh, w.par, w.g, w.i, vy);
        cx<double> back[4];
        ld4<PY, double>(y, Vh, w.par, w.g, w.i, back);
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[0] += back[k].re * back[k].re + back[k].im * back[k].im;
    }
};

// CG step: x += alpha p ; r -= alpha w ; |r|^2   (alpha read from device scalars)
template <int PX, int P>
struct CgStep {
    static constexpr int NS = 1;
    void* x;
    const void* p;
    void* r;
    const void* w;
    const double* sc;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        using R = typename Traits<P>::real;
        const R a = (R)sc[S_ALPHA];
        // a zero or non-finite step length leaves the iterate as it was, so that a solve that
        // runs into a non-finite value still holds its last finite iterate
        const bool move = a != (R)0 && isfinite(a);
        cx<R> vx[4], vp[4], vr[4], vw[4];
        ld4<P, R>(p, Vh, u.par, u.g, u.i, vp);
        ld4<P, R>(r, Vh, u.par, u.g, u.i, vr);
        ld4<P, R>(w, Vh, u.par, u.g, u.i, vw);
        if (move) {
            ld4<PX, R>(x, Vh, u.par, u.g, u.i, vx);
#pragma unroll
            for (int k = 0; k < 4; ++k) vx[k] = vx[k] + scale(vp[k], a);
            st4<PX, R>(x, Vh, u.par, u.g, u.i, vx);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) vr[k] = vr[k] - scale(vw[k], a);
        st4<P, R>(r, Vh, u.par, u.g, u.i, vr);
        // reduce what is stored (rounded to P), in FP64; FP64 stores the values as they are
        cx<double> back[4];
        if constexpr (P == F64) {
#pragma unroll
            for (int k = 0; k < 4; ++k) back[k] = {(double)vr[k].re, (double)vr[k].im};
        } else {
            ld4<P, double>(r, Vh, u.par, u.g, u.i, back);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[0] += back[k].re * back[k].re + back[k].im * back[k].im;
    }
};

// p = r + beta p   (beta read from device scalars)
template <int P>
struct CgDirection {
    static constexpr int NS = 0;
    const void* r;
    void* p;
    const double* sc;
    int Vh;
    __device__ void operator()(const Unit& u, double*) const
    {
        using R = typename Traits<P>::real;
        const R b = (R)sc[S_BETA];
        cx<R> vr[4], vp[4];
        ld4<P, R>(r, Vh, u.par, u.g, u.i, vr);
        ld4<P, R>(p, Vh, u.par, u.g, u.i, vp);
#pragma unroll
        for (int k = 0; k < 4; ++k) vp[k] = vr[k] + scale(vp[k], b);
        st4<P, R>(p, Vh, u.par, u.g, u.i, vp);
    }
};

// r = eta - t ; |r|^2   (all FP64)
struct Residual {
    static constexpr int NS = 1;
    const void* eta;
    const void* t;
    void* r;
    int Vh;
    __device__ void operator()(const Unit& u, double* acc) const
    {
        cx<double> ve[4], vt[4];
        ld4<F64, double>(eta, Vh, u.par, u.g, u.i, ve);
        ld4<F64, double>(t, Vh, u.par, u.g, u.i, vt);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ve[k] = ve[k] - vt[k];
            acc[0] += ve[k].re * ve[k].re + ve[k].im * ve[k].im;
        }
        st4<F64, double>(r, Vh, u.par, u.g, u.i, ve);
    }
};

// x_hi += s x_lo ; x_lo = 0
template <int PL>
struct Accumulate {
    static constexpr int NS = 0;
    void* xhi;
    void* xlo;
    double s;
    int Vh;
    __device__ void operator()(const Unit& u, double*) const
    {
        cx<double> vh[4], vl[4];
        ld4<F64, double>(xhi, Vh, u.par, u.g, u.i, vh);
        ld4<PL, double>(xlo, Vh, u.par, u.g, u.i, vl);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            vh[k] = vh[k] + scale(vl[k], s);
            vl[k] = {0.0, 0.0};
        }
        st4<F64, double>(xhi, Vh, u.par, u.g, u.i, vh);
        st4<PL, double>(xlo, Vh, u.par, u.g, u.i, vl);
    }
};

// x = 0
template <int P>
struct Zero {
    static constexpr int NS = 0;
    void* x;
    int Vh;
    __device__ void operator()(const Unit& u, double*) const
    {
        cx<double> v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        st4<P, double>(x, Vh, u.par, u.g, u.i, v);
    }
};

// ---------------------------------------------------------------- host helpers

int dw_launch(qdw_op* op, const void* in, void* out, int prec, bool dag, hipStream_t st);
// the even-odd reduced operator on the even half of in (odd half of out: scratch)
int schur_launch(qdw_op* op, const void* in, void* out, int prec, bool dag, hipStream_t st);

// read `n` device doubles at `src` (synchronises the stream)
inline int read_device(const qdw_op* op, const double* src, int n, double* out, hipStream_t st)
{
    QDW_CHECK(n >= 1 && n <= kHostScalars, QDW_EINVAL, "internal: read-back too large");
    QDW_HIP(hipMemcpyAsync(op->host_scalars, src, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    QDW_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < n; ++k) out[k] = op->host_scalars[k];
    return QDW_OK;
}

// read `n` device scalars starting at `slot` (synchronises the stream)
inline int read_scalars(const qdw_op* op, int slot, int n, double* out, hipStream_t st)
{
    QDW_HIP(hipMemcpyAsync(op->host_scalars, op->scalars + slot, sizeof(double) * n,
                           hipMemcpyDeviceToHost, st));
    QDW_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < n; ++k) out[k] = op->host_scalars[k];
    return QDW_OK;
}

}  // namespace qdw
