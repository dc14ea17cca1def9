// qdw_internal.h -- device-side building blocks shared by the HIP kernels of libqdw.
//
// Layout ("eo-SoA"): every per-site field is split by site parity (even sites first,
// as in the paper's even-odd ordered operator, Sec. 3 / Fig. 3 left) and stored as
// [parity][site/64][chunk][site%64] where a chunk is 16 bytes of one site's data (see
// chunk_at). Consecutive lanes of a wavefront read consecutive 16-byte chunks: one
// fully coalesced 1 KiB transaction per wave per chunk.
//
//   spinor  24 reals/site  (12 complex, index spin*3 + colour)
//           F64: 12 chunks (1 complex each), F32: 6 (2 complex), F16/BF16: 3 (4 complex)
//   link    rows 0 and 1 of the U(3) link U = exp(i theta) V (6 complex) and its
//           determinant d = exp(3 i theta), per direction mu
//           F64: 6 chunks + a separate array of d (8 B, encode_phase), F32: 3 chunks +
//           d array (8 B),
//           F16/BF16: 2 chunks = the 6 complex and d
//           The third row is rebuilt in registers as d conj(row0 x row1).
//   clover  2 chirality blocks x 36 reals (6 real diagonal, 15 complex upper triangle,
//           row-major), (4 + m0) included. F64: 36 chunks, F32: 18, F16/BF16: 9.
//           The D kernels read the compact form instead (54 reals, dirac_core.h).
//
// The even-odd index of a site is lex/2 with lex = ((x0*L1 + x1)*L2 + x2)*L3 + x3;
// this is a bijection per parity because L3 is even.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace qdw {

enum Prec { F64 = 0, F32 = 1, F16S = 2, BF16S = 3 };

struct Geom {
    int L[4];      // T, L1, L2, L3 (direction 0 is time)
    int stride[4]; // lexicographic strides
    int V, Vh;
    int bc_t;      // -1 antiperiodic, +1 periodic in time
    double cdiag;  // 4 + m0, the constant diagonal of the clover term
    int S;         // even-odd sites per time slice and parity (L1*L2*L3/2)
    int ts;        // sites per parity of a site-kernel workgroup (64 or 128; 2*ts lanes)
    int ntile;     // workgroups per time slice
    int nt;        // time slices per chunk of the workgroup walk (a divisor of T, <= 64)
    int walk;      // workgroup order within a chunk (walk_site)
    int slab;      // even-odd sites per parity of one x1 slab of a time slice (L2*L3/2)
    int tps;       // ts-site tiles per slab (walk 1)
};

// set the walk of the site kernels (ts, nt, walk as in walk_site)
inline void set_walk(Geom& g, int ts, int nt, int walk)
{
    g.ts = ts;
    g.nt = nt;
    g.walk = walk;
    g.slab = g.L[2] * g.L[3] / 2;
    g.tps = (g.slab + ts - 1) / ts;
    g.ntile = walk ? g.L[1] * g.tps : (g.S + ts - 1) / ts;
}

// ---------------------------------------------------------------- scalar types

struct bf16_t { uint16_t bits; };

__host__ __device__ inline float bf16_to_float(uint16_t b)
{
    union { uint32_t u; float f; } v;
    v.u = ((uint32_t)b) << 16;
    return v.f;
}

// round to nearest even; NaN stays NaN
__host__ __device__ inline uint16_t float_to_bf16(float f)
{
    union { uint32_t u; float f; } v;
    v.f = f;
    if ((v.u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((v.u >> 16) | 0x40);
    uint32_t lsb = (v.u >> 16) & 1u;
    v.u += 0x7fffu + lsb;
    return (uint16_t)(v.u >> 16);
}

template <int P> struct Traits;
template <> struct Traits<F64> {
    using real = double;     // arithmetic type
    using store = double;    // storage scalar
    static constexpr int SPIN_CHUNKS = 12, LINK_CHUNKS = 6, CLOVER_CHUNKS = 36;
    static constexpr int PER_CHUNK = 2;   // reals per 16-byte chunk
};
template <> struct Traits<F32> {
    using real = float;
    using store = float;
    static constexpr int SPIN_CHUNKS = 6, LINK_CHUNKS = 3, CLOVER_CHUNKS = 18;
    static constexpr int PER_CHUNK = 4;
};
template <> struct Traits<F16S> {
    using real = float;
    using store = _Float16;
    static constexpr int SPIN_CHUNKS = 3, LINK_CHUNKS = 2, CLOVER_CHUNKS = 9;
    static constexpr int PER_CHUNK = 8;
};
template <> struct Traits<BF16S> {
    using real = float;
    using store = uint16_t;
    static constexpr int SPIN_CHUNKS = 3, LINK_CHUNKS = 2, CLOVER_CHUNKS = 9;
    static constexpr int PER_CHUNK = 8;
};

template <int P> __device__ __forceinline__ typename Traits<P>::real to_real(typename Traits<P>::store s);
template <> __device__ __forceinline__ double to_real<F64>(double s) { return s; }
template <> __device__ __forceinline__ float to_real<F32>(float s) { return s; }
template <> __device__ __forceinline__ float to_real<F16S>(_Float16 s) { return (float)s; }
template <> __device__ __forceinline__ float to_real<BF16S>(uint16_t s) { return bf16_to_float(s); }

template <int P> __device__ __forceinline__ typename Traits<P>::store to_store(typename Traits<P>::real r);
template <> __device__ __forceinline__ double to_store<F64>(double r) { return r; }
template <> __device__ __forceinline__ float to_store<F32>(float r) { return r; }
template <> __device__ __forceinline__ _Float16 to_store<F16S>(float r) { return (_Float16)r; }
template <> __device__ __forceinline__ uint16_t to_store<BF16S>(float r) { return float_to_bf16(r); }

// One 16-byte chunk, viewed as PER_CHUNK storage scalars.
template <int P> struct Chunk {
    typename Traits<P>::store v[Traits<P>::PER_CHUNK];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int P>
__device__ __forceinline__ Chunk<P> load_chunk(const void* base, long idx)
{
    const u32x4 raw = __builtin_nontemporal_load((const u32x4*)base + idx);
    Chunk<P> c;
    __builtin_memcpy(&c, &raw, 16);
    return c;
}

template <int P>
__device__ __forceinline__ Chunk<P> load_chunk_cached(const void* base, long idx)
{
    const u32x4 raw = ((const u32x4*)base)[idx];
    Chunk<P> c;
    __builtin_memcpy(&c, &raw, 16);
    return c;
}

// ---------------------------------------------------------------- AoSoA addressing
//
// A per-site field is stored in rows (a parity, or parity*4 + mu for links); a row holds
// its sites in blocks of kSB = 64 consecutive even-odd indices, and a block stores chunk 0
// of its 64 sites, then chunk 1, ...: [row][site/64][chunk][site%64]. A wavefront's 64
// lanes read one contiguous 1 KiB run per chunk, and all chunks of one site lie within
// one block of NC KiB (a few pages at most), which keeps address translation cheap.
constexpr int kSB = 64;

__host__ __device__ __forceinline__ int padded(int Vh) { return (Vh + kSB - 1) & ~(kSB - 1); }

__host__ __device__ __forceinline__ long chunk_at(int Vh, int NC, int row, int k, int i)
{
    const unsigned u = (unsigned)i;
    return (((long)row * (padded(Vh) / kSB) + (u / kSB)) * NC + k) * kSB + (u % kSB);
}

template <int P>
__device__ __forceinline__ void store_chunk(void* base, long idx, const Chunk<P>& c)
{
    u32x4 raw;
    __builtin_memcpy(&raw, &c, 16);
    __builtin_nontemporal_store(raw, (u32x4*)base + idx);
}

// ---------------------------------------------------------------- complex helpers

template <typename R> struct cx { R re, im; };

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return {a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> cmul_conj(cx<R> a, cx<R> b)   // conj(a) * b
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ cx<R> conj_(cx<R> a) { return {a.re, -a.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }

// Fused multiply-adds, written out so that every complex multiply-accumulate is four FMA
// instructions (a product followed by an addition otherwise often stays a multiply and an
// add): c + a b and c + conj(a) b.
template <typename R> __device__ __forceinline__ R fmar(R a, R b, R c);
template <> __device__ __forceinline__ float fmar<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmar<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename R> __device__ __forceinline__ cx<R> cmadd(cx<R> c, cx<R> a, cx<R> b)
{
    return {fmar(a.re, b.re, fmar(-a.im, b.im, c.re)), fmar(a.re, b.im, fmar(a.im, b.re, c.im))};
}
template <typename R> __device__ __forceinline__ cx<R> cmadd_conj(cx<R> c, cx<R> a, cx<R> b)
{
    return {fmar(a.re, b.re, fmar(a.im, b.im, c.re)), fmar(a.re, b.im, fmar(-a.im, b.re, c.im))};
}
template <typename R> __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.re * s, a.im * s}; }

// ---------------------------------------------------------------- field access

// spinor of one site (12 complex) from an eo-SoA field
template <int P>
__device__ __forceinline__ void load_spinor(const void* f, int Vh, int par, int i,
                                            cx<typename Traits<P>::real> s[12])
{
    using T = Traits<P>;
    const long base = chunk_at(Vh, T::SPIN_CHUNKS, par, 0, i);
#pragma unroll
    for (int k = 0; k < T::SPIN_CHUNKS; ++k) {
        Chunk<P> c = load_chunk_cached<P>(f, base + (long)k * kSB);
#pragma unroll
        for (int j = 0; j < T::PER_CHUNK / 2; ++j)
            s[k * (T::PER_CHUNK / 2) + j] = {to_real<P>(c.v[2 * j]), to_real<P>(c.v[2 * j + 1])};
    }
}

template <int P>
__device__ __forceinline__ void store_spinor(void* f, int Vh, int par, int i,
                                             const cx<typename Traits<P>::real> s[12])
{
    using T = Traits<P>;
    const long base = chunk_at(Vh, T::SPIN_CHUNKS, par, 0, i);
#pragma unroll
    for (int k = 0; k < T::SPIN_CHUNKS; ++k) {
        Chunk<P> c;
#pragma unroll
        for (int j = 0; j < T::PER_CHUNK / 2; ++j) {
            c.v[2 * j] = to_store<P>(s[k * (T::PER_CHUNK / 2) + j].re);
            c.v[2 * j + 1] = to_store<P>(s[k * (T::PER_CHUNK / 2) + j].im);
        }
        store_chunk<P>(f, base + (long)k * kSB, c);
    }
}

// site coordinates of (parity, eo index)
__device__ __forceinline__ void eo_coords(const Geom& g, int par, int i, int x[4], int& lex)
{
    int l = 2 * i;
    int r = l / g.L[3];
    x[3] = l - r * g.L[3];
    int r2 = r / g.L[2];
    x[2] = r - r2 * g.L[2];
    int r3 = r2 / g.L[1];
    x[1] = r2 - r3 * g.L[1];
    x[0] = r3;
    if (((x[0] + x[1] + x[2] + x[3]) & 1) != par) { x[3] += 1; l += 1; }
    lex = l;
}

// lexicographic index of the neighbour x +- mu, given x's coordinates and lex index
__device__ __forceinline__ int lex_fwd(const Geom& g, const int x[4], int lex, int mu)
{
    return (x[mu] == g.L[mu] - 1) ? lex - (g.L[mu] - 1) * g.stride[mu] : lex + g.stride[mu];
}
__device__ __forceinline__ int lex_bwd(const Geom& g, const int x[4], int lex, int mu)
{
    return (x[mu] == 0) ? lex + (g.L[mu] - 1) * g.stride[mu] : lex - g.stride[mu];
}

// XCD-aware block mapping: hardware hands out workgroups round-robin over the 8 XCDs;
// remap so that each XCD walks one contiguous range of tiles and neighbouring tiles
// share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblk)
{
    const int q = nblk >> 3, r = nblk & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Workgroup walk of the site kernels: a workgroup handles ts sites of one time slice in
// both parities (2*ts lanes, T * ntile workgroups). Logical workgroups are grouped in
// chunks of nt time slices; within a chunk:
//   walk 0: tiles of ts consecutive even-odd indices of a slice; the nt slices of one tile
//           are consecutive, then the next tile. The t +- 1 neighbours are loaded by
//           workgroups running at the same time; the x1 +- 1 neighbours, L2*L3/(2 ts)
//           tiles away, by workgroups about nt times that many positions away.
//   walk 1: each x1 slab of a slice (L2*L3/2 sites per parity) is cut into tiles of ts
//           sites (x2 rows); for one tile position the nt slices and then all L1 slabs
//           are consecutive, so the t and the x1 neighbours are both loaded by workgroups
//           a few positions away, and only the x2 neighbours across a tile edge are far.
// Logical workgroups map XCD-contiguously (xcd_tile), so neighbours in this order share
// an XCD and its L2. Shapes are chosen per lattice by the autotuner. Returns false for the
// lanes of a ragged last tile; `par` and the lane come from the thread index.
__device__ __forceinline__ bool walk_site(const Geom& g, int logical, int tid, int& par, int& i)
{
    par = tid >= g.ts ? 1 : 0;
    const int lane = tid - par * g.ts;
    const int per_chunk = g.nt * g.ntile;
    const int c = logical / per_chunk;
    const int r = logical - c * per_chunk;
    if (g.walk == 0) {
        const int s = r / g.nt;
        const int t = c * g.nt + (r - s * g.nt);
        const int k = s * g.ts + lane;
        i = t * g.S + k;
        return k < g.S;
    }
    const int per_b = g.nt * g.L[1];
    const int b = r / per_b;
    const int r2 = r - b * per_b;
    const int x1 = r2 / g.nt;
    const int t = c * g.nt + (r2 - x1 * g.nt);
    const int k = b * g.ts + lane;
    i = t * g.S + x1 * g.slab + k;
    return k < g.slab;
}

inline int walk_blocks(const Geom& g) { return g.L[0] * g.ntile; }

// Several right-hand sides of one lattice in one launch, the right-hand side the fastest-
// varying workgroup index (the workgroups of one tile or block for all of them run side by
// side and share its links and clover through L2): their fields sit at a fixed byte stride,
// and gate[r * gstride] == 0 marks a finished one, whose workgroups return at once. The
// default is a single field and no gate.
struct RhsStride {
    long fstride = 0;
    const int* gate = nullptr;
    int gstride = 0;
    int nrhs = 1;
};

}  // namespace qdw
