// op.hip -- operator set-up: link compression, clover term, precision copies, spinor
// pack/unpack, and the error plumbing of the C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "qdw_host.h"
#include "dirac_core.h"

using namespace qdw;

namespace qdw {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace qdw

extern "C" const char* qdw_last_error(void) { return qdw::g_last_error.c_str(); }

namespace {

// ------------------------------------------------------------------ canonical links

struct M3 { cx<double> a[9]; };

__device__ inline M3 mat_mul(const M3& x, const M3& y)
{
    M3 z;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = s + x.a[i * 3 + k] * y.a[k * 3 + j];
            z.a[i * 3 + j] = s;
        }
    return z;
}

// x * y^+
__device__ inline M3 mat_mul_dag(const M3& x, const M3& y)
{
    M3 z;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = s + x.a[i * 3 + k] * conj_(y.a[j * 3 + k]);
            z.a[i * 3 + j] = s;
        }
    return z;
}

__device__ inline M3 dag(const M3& x)
{
    M3 z;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) z.a[i * 3 + j] = conj_(x.a[j * 3 + i]);
    return z;
}

// full U(3) link exp(i theta) V at lexicographic site `lex`, direction mu
__device__ inline M3 link_u3(const double* su3, const double* theta, long lex, int mu)
{
    M3 m;
    const double* p = su3 + ((lex * 4 + mu) * 9) * 2;
    double s, c;
    sincos(theta[lex * 4 + mu], &s, &c);
    const cx<double> ph = {c, s};
#pragma unroll
    for (int k = 0; k < 9; ++k) m.a[k] = ph * cx<double>{p[2 * k], p[2 * k + 1]};
    return m;
}

__device__ inline long lex_of(const Geom& g, const int x[4])
{
    return ((long)(x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}

__device__ inline long shifted(const Geom& g, const int x[4], int mu, int dmu, int nu, int dnu)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + dmu + g.L[mu]) % g.L[mu];
    y[nu] = (y[nu] + dnu + g.L[nu]) % g.L[nu];
    return lex_of(g, y);
}

// ------------------------------------------------------------------ unitarity check

// *p = 0 (a kernel, not a memset node, so the set-up can be captured)
__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

__global__ void unitarity_kernel(const double* su3, long nlinks, unsigned long long* worst)
{
    __shared__ double red[256];
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double dev = 0.0;
    if (l < nlinks) {
        M3 m;
        const double* p = su3 + l * 18;
        bool finite = true;
        for (int k = 0; k < 9; ++k) {
            m.a[k] = {p[2 * k], p[2 * k + 1]};
            finite = finite && isfinite(p[2 * k]) && isfinite(p[2 * k + 1]);
        }
        M3 e = mat_mul_dag(m, m);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                cx<double> d = e.a[i * 3 + j];
                if (i == j) d.re -= 1.0;
                dev = fmax(dev, fmax(fabs(d.re), fabs(d.im)));
            }
        // det = row0 . (row1 x row2)
        cx<double> c0 = m.a[4] * m.a[8] - m.a[5] * m.a[7];
        cx<double> c1 = m.a[5] * m.a[6] - m.a[3] * m.a[8];
        cx<double> c2 = m.a[3] * m.a[7] - m.a[4] * m.a[6];
        cx<double> det = m.a[0] * c0 + m.a[1] * c1 + m.a[2] * c2;
        dev = fmax(dev, fmax(fabs(det.re - 1.0), fabs(det.im)));
        if (!finite) dev = 1e300;
    }
    red[threadIdx.x] = dev;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    // non-negative doubles order like their bit patterns
    if (threadIdx.x == 0) atomicMax(worst, (unsigned long long)__double_as_longlong(red[0]));
}

// ------------------------------------------------------------------ link compression

// A stored link is rows 0 and 1 of the full U(3) matrix U = exp(i theta) V and the phase
// d = det U = exp(3 i theta): row 2 of U is d * conj(row0 x row1), since row 2 of V is
// conj(v0 x v1) and u0 x u1 = exp(2 i theta) v0 x v1. No trigonometry at apply time.
__global__ void pack_links_kernel(Geom g, const double* su3, const double* theta, void* l64,
                                  void* d64, void* l32, void* d32, void* l16, void* lb16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    const int mu = blockIdx.z;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const double* p = su3 + (((long)lex * 4 + mu) * 9) * 2;  // rows 0 and 1: 12 reals
    const double th = theta[(long)lex * 4 + mu];
    const long row = (long)(par * 4 + mu);
    double s1, c1, s3, c3;
    sincos(th, &s1, &c1);
    sincos(3.0 * th, &s3, &c3);
    double r[12];
    for (int k = 0; k < 6; ++k) {  // r = exp(i theta) * (rows 0, 1 of V)
        const double a = p[2 * k], b = p[2 * k + 1];
        r[2 * k] = c1 * a - s1 * b;
        r[2 * k + 1] = c1 * b + s1 * a;
    }
    // FP64: 6 chunks of one complex each, d in one double (encode_phase)
    for (int k = 0; k < 6; ++k) {
        double2 v = {r[2 * k], r[2 * k + 1]};
        ((double2*)l64)[chunk_at(g.Vh, 6, (int)row, k, i)] = v;
    }
    ((double*)d64)[row * g.Vh + i] = encode_phase(c3, s3);
    // FP32: 3 chunks of two complex each, d as a float2 array
    for (int k = 0; k < 3; ++k) {
        float4 v = {(float)r[4 * k], (float)r[4 * k + 1], (float)r[4 * k + 2], (float)r[4 * k + 3]};
        ((float4*)l32)[chunk_at(g.Vh, 3, (int)row, k, i)] = v;
    }
    ((float2*)d32)[row * g.Vh + i] = float2{(float)c3, (float)s3};
    // FP16 / BF16: 12 reals, then d, then two zeros
    double e[16];
    for (int k = 0; k < 12; ++k) e[k] = r[k];
    e[12] = c3; e[13] = s3; e[14] = 0.0; e[15] = 0.0;
    _Float16* h = (_Float16*)l16;
    uint16_t* b = (uint16_t*)lb16;
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 8; ++j) {
            const long at = chunk_at(g.Vh, 2, (int)row, k, i) * 8 + j;
            h[at] = (_Float16)e[8 * k + j];
            b[at] = float_to_bf16((float)e[8 * k + j]);
        }
}

// ------------------------------------------------------------------ clover term

// Fhat_{mu nu}(x) = (Q - Q^+)/8, Q = sum of the four counter-clockwise leaves at x.
__device__ M3 field_strength(const Geom& g, const double* su3, const double* theta,
                             const int x[4], long lex, int mu, int nu)
{
    const long xpm = shifted(g, x, mu, 1, nu, 0), xpn = shifted(g, x, mu, 0, nu, 1);
    const long xmm = shifted(g, x, mu, -1, nu, 0), xmn = shifted(g, x, mu, 0, nu, -1);
    const long xmm_pn = shifted(g, x, mu, -1, nu, 1), xmm_mn = shifted(g, x, mu, -1, nu, -1);
    const long xmn_pm = shifted(g, x, mu, 1, nu, -1);
    const M3 umu = link_u3(su3, theta, lex, mu), unu = link_u3(su3, theta, lex, nu);
    const M3 umu_mm = link_u3(su3, theta, xmm, mu), unu_mm = link_u3(su3, theta, xmm, nu);
    const M3 umu_mn = link_u3(su3, theta, xmn, mu), unu_mn = link_u3(su3, theta, xmn, nu);
    // (x, x+mu, x+mu+nu, x+nu)
    M3 q = mat_mul_dag(mat_mul_dag(mat_mul(umu, link_u3(su3, theta, xpm, nu)),
                                   link_u3(su3, theta, xpn, mu)), unu);
    // (x, x+nu, x-mu+nu, x-mu)
    M3 t = mat_mul(mat_mul_dag(mat_mul_dag(unu, link_u3(su3, theta, xmm_pn, mu)), unu_mm), umu_mm);
    for (int k = 0; k < 9; ++k) q.a[k] = q.a[k] + t.a[k];
    // (x, x-mu, x-mu-nu, x-nu)
    t = mat_mul(mat_mul(mat_mul_dag(dag(umu_mm), link_u3(su3, theta, xmm_mn, nu)),
                        link_u3(su3, theta, xmm_mn, mu)), unu_mn);
    for (int k = 0; k < 9; ++k) q.a[k] = q.a[k] + t.a[k];
    // (x, x-nu, x-nu+mu, x+mu)
    t = mat_mul_dag(mat_mul(mat_mul(dag(unu_mn), umu_mn), link_u3(su3, theta, xmn_pm, nu)), umu);
    for (int k = 0; k < 9; ++k) q.a[k] = q.a[k] + t.a[k];
    M3 f;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cx<double> a = q.a[i * 3 + j], b = conj_(q.a[j * 3 + i]);
            f.a[i * 3 + j] = scale(a - b, 0.125);
        }
    return f;
}

// A_+-(x) = (4 + m0) + (i csw/2) [[E3, E1 - i E2], [E1 + i E2, -E3]] with
// E1 = +-F01 - F23, E2 = +-F02 + F13, E3 = +-F03 - F12 (chiral basis:
// sigma_0k = diag(s_k, -s_k), sigma_12 = -s_3, sigma_13 = s_2, sigma_23 = -s_1).
__global__ void clover_kernel(Geom g, const double* su3, const double* theta, double m0,
                              double csw, double2* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const M3 f01 = field_strength(g, su3, theta, x, lex, 0, 1);
    const M3 f02 = field_strength(g, su3, theta, x, lex, 0, 2);
    const M3 f03 = field_strength(g, su3, theta, x, lex, 0, 3);
    const M3 f12 = field_strength(g, su3, theta, x, lex, 1, 2);
    const M3 f13 = field_strength(g, su3, theta, x, lex, 1, 3);
    const M3 f23 = field_strength(g, su3, theta, x, lex, 2, 3);
    double reals[72];
    for (int blk = 0; blk < 2; ++blk) {
        const double s = blk == 0 ? 1.0 : -1.0;
        cx<double> S[2][2][9];
        for (int k = 0; k < 9; ++k) {
            cx<double> e1 = scale(f01.a[k], s) - f23.a[k];
            cx<double> e2 = scale(f02.a[k], s) + f13.a[k];
            cx<double> e3 = scale(f03.a[k], s) - f12.a[k];
            S[0][0][k] = e3;
            S[0][1][k] = e1 - times_i(e2);
            S[1][0][k] = e1 + times_i(e2);
            S[1][1][k] = scale(e3, -1.0);
        }
        // entry (r, c) of the 6x6 block, r = a*3 + i, c = b*3 + j
        auto entry = [&](int r, int c) {
            const int a = r / 3, ii = r % 3, b = c / 3, jj = c % 3;
            cx<double> v = scale(times_i(S[a][b][ii * 3 + jj]), 0.5 * csw);
            if (r == c) v.re += 4.0 + m0;
            return v;
        };
        double* o = reals + 36 * blk;
        for (int r = 0; r < 6; ++r) o[r] = entry(r, r).re;
        int n = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c) {
                cx<double> v = entry(r, c);
                o[6 + 2 * n] = v.re;
                o[6 + 2 * n + 1] = v.im;
                ++n;
            }
    }
    for (int k = 0; k < 36; ++k)
        out[chunk_at(g.Vh, 36, par, k, i)] = double2{reals[2 * k], reals[2 * k + 1]};
}

// The inverse of each 6x6 Hermitian chirality block of the clover term (for the even-odd
// reduced operator): Gauss-Jordan elimination with partial pivoting in FP64, stored in the
// clover term's packed Hermitian format (6 diagonal reals, then the upper triangle row by
// row). A singular block leaves non-finite entries, which a solve reports as status -3.
__global__ void clover_inv_kernel(Geom g, const double2* clov, double2* inv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    double in[72], outr[72];
    for (int k = 0; k < 36; ++k) {
        const double2 v = clov[chunk_at(g.Vh, 36, par, k, i)];
        in[2 * k] = v.x;
        in[2 * k + 1] = v.y;
    }
    for (int blk = 0; blk < 2; ++blk) {
        const double* a = in + 36 * blk;
        cx<double> m[6][6], r[6][6];
        int n = 0;
        for (int u = 0; u < 6; ++u) {
            m[u][u] = {a[u], 0.0};
            for (int v = u + 1; v < 6; ++v) {
                m[u][v] = {a[6 + 2 * n], a[6 + 2 * n + 1]};
                m[v][u] = {a[6 + 2 * n], -a[6 + 2 * n + 1]};
                ++n;
            }
        }
        for (int u = 0; u < 6; ++u)
            for (int v = 0; v < 6; ++v) r[u][v] = {u == v ? 1.0 : 0.0, 0.0};
        for (int c = 0; c < 6; ++c) {
            int pv = c;
            double best = m[c][c].re * m[c][c].re + m[c][c].im * m[c][c].im;
            for (int u = c + 1; u < 6; ++u) {
                const double mag = m[u][c].re * m[u][c].re + m[u][c].im * m[u][c].im;
                if (mag > best) {
                    best = mag;
                    pv = u;
                }
            }
            if (pv != c)
                for (int v = 0; v < 6; ++v) {
                    const cx<double> t = m[c][v];
                    m[c][v] = m[pv][v];
                    m[pv][v] = t;
                    const cx<double> w = r[c][v];
                    r[c][v] = r[pv][v];
                    r[pv][v] = w;
                }
            const double n2 = m[c][c].re * m[c][c].re + m[c][c].im * m[c][c].im;
            const cx<double> piv = {m[c][c].re / n2, -m[c][c].im / n2};  // 1 / m_cc
            for (int v = 0; v < 6; ++v) {
                m[c][v] = m[c][v] * piv;
                r[c][v] = r[c][v] * piv;
            }
            for (int u = 0; u < 6; ++u) {
                if (u == c) continue;
                const cx<double> f = m[u][c];
                for (int v = 0; v < 6; ++v) {
                    m[u][v] = m[u][v] - f * m[c][v];
                    r[u][v] = r[u][v] - f * r[c][v];
                }
            }
        }
        double* o = outr + 36 * blk;
        for (int u = 0; u < 6; ++u) o[u] = r[u][u].re;
        n = 0;
        for (int u = 0; u < 6; ++u)
            for (int v = u + 1; v < 6; ++v) {
                o[6 + 2 * n] = r[u][v].re;
                o[6 + 2 * n + 1] = r[u][v].im;
                ++n;
            }
    }
    for (int k = 0; k < 36; ++k)
        inv[chunk_at(g.Vh, 36, par, k, i)] = double2{outr[2 * k], outr[2 * k + 1]};
}

// FP64 eo-SoA array of `nr` reals per site -> lower precision copies
__global__ void convert_site_reals(Geom g, int nr, const double* src, float* f32, _Float16* f16,
                                   uint16_t* b16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    for (int q = 0; q < nr; ++q) {
        const double v = src[chunk_at(g.Vh, nr / 2, par, q / 2, i) * 2 + q % 2];
        f32[chunk_at(g.Vh, nr / 4, par, q / 4, i) * 4 + q % 4] = (float)v;
        const long a16 = chunk_at(g.Vh, nr / 8, par, q / 8, i) * 8 + q % 8;
        f16[a16] = (_Float16)v;
        b16[a16] = float_to_bf16((float)v);
    }
}

// The compact form of the clover blocks that the D kernels read (see clover54_apply):
// per chirality block, H = (a - d) / 2 and b, where a, d are the colour blocks of its two
// spins on the diagonal (a + d = 2 (4 + m0) 1 in the chiral basis) and b the colour block
// between them; then rounded to the lower precisions.
__global__ void compact_clover_kernel(Geom g, const double2* cl, double2* c64, float* c32,
                                      _Float16* c16, uint16_t* cb16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    double a[72];
    for (int k = 0; k < 36; ++k) {
        const double2 v = cl[chunk_at(g.Vh, 36, par, k, i)];
        a[2 * k] = v.x;
        a[2 * k + 1] = v.y;
    }
    // entry (r, q), r < q, of the 6x6 block starting at a + 36 blk (row-major upper triangle)
    auto up = [&](int blk, int r, int q, int part) {
        const int n = r * 6 - r * (r + 1) / 2 + (q - r - 1);
        return a[36 * blk + 6 + 2 * n + part];
    };
    double o[56];
    for (int blk = 0; blk < 2; ++blk) {
        double* hd = o + 3 * blk;
        double* hu = o + (blk ? 30 : 6);
        double* b = o + (blk ? 36 : 12);
        for (int r = 0; r < 3; ++r) hd[r] = 0.5 * (a[36 * blk + r] - a[36 * blk + 3 + r]);
        const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int e = 0; e < 3; ++e)
            for (int part = 0; part < 2; ++part)
                hu[2 * e + part] = 0.5 * (up(blk, pr[e][0], pr[e][1], part) -
                                          up(blk, 3 + pr[e][0], 3 + pr[e][1], part));
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q)
                for (int part = 0; part < 2; ++part) b[2 * (3 * r + q) + part] = up(blk, r, 3 + q, part);
    }
    o[54] = o[55] = 0.0;
    for (int k = 0; k < 27; ++k) c64[chunk_at(g.Vh, 27, par, k, i)] = double2{o[2 * k], o[2 * k + 1]};
    for (int q = 0; q < 56; ++q) {
        c32[chunk_at(g.Vh, 14, par, q / 4, i) * 4 + q % 4] = (float)o[q];
        const long a16 = chunk_at(g.Vh, 7, par, q / 8, i) * 8 + q % 8;
        c16[a16] = (_Float16)o[q];
        cb16[a16] = float_to_bf16((float)o[q]);
    }
}

// ------------------------------------------------------------------ spinor pack

template <int P>
__global__ void pack_kernel(Geom g, const double* can, void* eo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    using R = typename Traits<P>::real;
    cx<R> s[12];
    const double* p = can + (long)lex * 24;
    for (int k = 0; k < 12; ++k) s[k] = {(R)p[2 * k], (R)p[2 * k + 1]};
    store_spinor<P>(eo, g.Vh, par, i, s);
}

template <int P>
__global__ void unpack_kernel(Geom g, const void* eo, double* can)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    using R = typename Traits<P>::real;
    cx<R> s[12];
    load_spinor<P>(eo, g.Vh, par, i, s);
    double* p = can + (long)lex * 24;
    for (int k = 0; k < 12; ++k) {
        p[2 * k] = (double)s[k].re;
        p[2 * k + 1] = (double)s[k].im;
    }
}

// FP16 pack rounds each double once, straight to binary16 (no binary32 detour)
template <>
__global__ void pack_kernel<F16S>(Geom g, const double* can, void* eo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const double* p = can + (long)lex * 24;
    _Float16* h = (_Float16*)eo;
    for (int q = 0; q < 24; ++q)
        h[chunk_at(g.Vh, 3, par, q / 8, i) * 8 + q % 8] = (_Float16)p[q];
}

// FP64 pack straight from canonical doubles (no float detour)
template <>
__global__ void pack_kernel<F64>(Geom g, const double* can, void* eo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int par = blockIdx.y;
    if (i >= g.Vh) return;
    int x[4], lex;
    eo_coords(g, par, i, x, lex);
    const double* p = can + (long)lex * 24;
    for (int k = 0; k < 12; ++k)
        ((double2*)eo)[chunk_at(g.Vh, 12, par, k, i)] = double2{p[2 * k], p[2 * k + 1]};
}

// Byte offsets of the operator's arrays inside the caller's device block (each 256-byte
// aligned): compressed links and their determinants, clover blocks and their inverses in
// every precision, then the reduction scratch.
struct OpLayout {
    size_t links[4], det[4], clover[4], cloverinv[4], clover54[4], partials, scalars, worst,
        total;
};

OpLayout op_layout(int Vh)
{
    OpLayout L{};
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t at = off;
        off += (n + 255) & ~(size_t)255;
        return at;
    };
    const size_t nl = (size_t)padded(Vh) * 8;  // link slots per array (2 parities x 4 dirs)
    const size_t ns = (size_t)padded(Vh) * 2;  // site slots of both parities
    L.links[F64] = take(nl * 6 * 16);
    L.det[F64] = take(nl * 8);
    L.links[F32] = take(nl * 3 * 16);
    L.det[F32] = take(nl * 8);
    L.links[F16S] = take(nl * 2 * 16);
    L.links[BF16S] = take(nl * 2 * 16);
    L.det[F16S] = L.det[BF16S] = (size_t)-1;  // kept inside the 16-bit link chunks
    const size_t creal[4] = {8, 4, 2, 2};
    for (int p = 0; p < 4; ++p) L.clover[p] = take(ns * 72 * creal[p]);
    for (int p = 0; p < 4; ++p) L.cloverinv[p] = take(ns * 72 * creal[p]);
    const size_t c54[4] = {27 * 16, 14 * 16, 7 * 16, 7 * 16};  // compact clover, bytes per site
    for (int p = 0; p < 4; ++p) L.clover54[p] = take(ns * c54[p]);
    L.partials = take(sizeof(double) * kMaxPartials * kMaxScalars);
    L.scalars = take(sizeof(double) * kMaxScalars);
    L.worst = take(sizeof(unsigned long long));
    L.total = off + 256;  // room to align the caller's pointer
    return L;
}

// lattice checks shared by the size query and qdw_create
int check_lattice(const qdw_lattice* lat)
{
    QDW_CHECK(lat, QDW_EINVAL, "qdw_create: null lattice");
    const int L[4] = {lat->T, lat->L1, lat->L2, lat->L3};
    for (int mu = 0; mu < 4; ++mu)
        QDW_CHECK(L[mu] >= 2 && L[mu] % 2 == 0, QDW_EINVAL,
                  "qdw_create: every lattice extent must be even and >= 2");
    QDW_CHECK(lat->bc_t == 1 || lat->bc_t == -1, QDW_EINVAL, "qdw_create: bc_t must be +1 or -1");
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    QDW_CHECK(V <= (1L << 30), QDW_EINVAL, "qdw_create: volume above 2^30 sites");
    return QDW_OK;
}

}  // namespace

extern "C" size_t qdw_op_device_bytes(const qdw_lattice* lat)
{
    if (check_lattice(lat)) return 0;
    const long V = (long)lat->T * lat->L1 * lat->L2 * lat->L3;
    return op_layout((int)(V / 2)).total;
}

extern "C" size_t qdw_op_host_bytes(void) { return sizeof(double) * kHostScalars; }

extern "C" int qdw_create(const qdw_lattice* lat, const double* su3, const double* theta,
                          double m0, double csw, void* dev_mem, size_t dev_bytes, void* host_mem,
                          size_t host_bytes, void* stream, qdw_op** out)
{
    QDW_CHECK(lat && su3 && theta && out && dev_mem && host_mem, QDW_EINVAL,
              "qdw_create: null argument");
    *out = nullptr;
    if (const int rc = check_lattice(lat)) return rc;
    const int L[4] = {lat->T, lat->L1, lat->L2, lat->L3};
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    const OpLayout lay = op_layout((int)(V / 2));
    QDW_CHECK(dev_bytes >= lay.total, QDW_EWORKSPACE,
              "qdw_create: device block smaller than qdw_op_device_bytes()");
    QDW_CHECK(host_bytes >= qdw_op_host_bytes(), QDW_EWORKSPACE,
              "qdw_create: host block smaller than qdw_op_host_bytes()");
    hipStream_t st = (hipStream_t)stream;

    qdw_op* op = new qdw_op();
    std::memset(op, 0, sizeof(*op));
    Geom& g = op->g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = L[mu];
    g.stride[3] = 1;
    g.stride[2] = L[3];
    g.stride[1] = L[3] * L[2];
    g.stride[0] = L[3] * L[2] * L[1];
    g.V = (int)V;
    g.Vh = (int)(V / 2);
    g.bc_t = lat->bc_t;
    g.cdiag = 4.0 + m0;
    g.S = L[1] * L[2] * L[3] / 2;
    {
        int nt = 1;
        for (int d = 1; d <= 8; ++d)
            if (L[0] % d == 0) nt = d;
        set_walk(g, 128, nt, 0);
    }
    {
        // default D-kernel shapes (qdw_autotune or qdw_set_dw_shape may change them).
        // FP64 and FP32: the marching form on 64-site tiles, with the longest walk chunk
        // (at most 32 slices, dividing T) that still gives 512 workgroups, two per CU, so
        // that they march side by side in one round
        const int ntile = (g.S + 63) / 64;
        int nt = 1;
        for (int d = 32; d >= 1; d /= 2)
            if (L[0] % d == 0 && (long)(L[0] / d) * ntile >= 512) {
                nt = d;
                break;
            }
        op->dw_shape[F64] = {64, nt, 0, 0, 1};
        op->dw_shape[F32] = {64, nt, 1, 0, 1};
        // half-precision storage: the plain form (one lane per site, four waves per SIMD)
        // on 128-site tiles in chunks of two slices (T is even)
        op->dw_shape[F16S] = {128, 2, 0, 0, 0};
        op->dw_shape[BF16S] = {128, 2, 0, 0, 0};
    }
    op->m0 = m0;
    op->csw = csw;
    (void)hipGetDevice(&op->device);

    // every array lives in the caller's blocks
    char* base = (char*)(((uintptr_t)dev_mem + 255) & ~(uintptr_t)255);
    for (int p = 0; p < 4; ++p) {
        op->links[p] = base + lay.links[p];
        op->det[p] = lay.det[p] == (size_t)-1 ? nullptr : base + lay.det[p];
        op->clover[p] = base + lay.clover[p];
        op->cloverinv[p] = base + lay.cloverinv[p];
        op->clover54[p] = base + lay.clover54[p];
    }
    op->partials = (double*)(base + lay.partials);
    op->scalars = (double*)(base + lay.scalars);
    op->host_scalars = (double*)host_mem;

    auto fail = [&](int code, const std::string& msg) {
        set_error(msg);
        delete op;
        return code;
    };
#define CREATE_HIP(call)                                                               \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(QDW_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

    // 1. unitarity of the SU(3) parts (the worst deviation as the bits of a non-negative
    //    double, so an integer maximum orders them)
    unsigned long long* worst = (unsigned long long*)(base + lay.worst);
    zero_u64_kernel<<<1, 1, 0, st>>>(worst);
    CREATE_HIP(hipGetLastError());
    const long nlinks = V * 4;
    unitarity_kernel<<<(unsigned)((nlinks + 255) / 256), 256, 0, st>>>(su3, nlinks, worst);
    CREATE_HIP(hipGetLastError());
    CREATE_HIP(hipMemcpyAsync(op->host_scalars, worst, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
    CREATE_HIP(hipStreamSynchronize(st));
    double wdev;
    std::memcpy(&wdev, op->host_scalars, sizeof(wdev));
    if (!(wdev <= 1e-10))
        return fail(QDW_ENOTUNITARY, "qdw_create: a link deviates from SU(3) by " +
                                         std::to_string(wdev));

    // 2. compressed links in every precision
    dim3 gl((g.Vh + 255) / 256, 2, 4);
    pack_links_kernel<<<gl, 256, 0, st>>>(g, su3, theta, op->links[F64], op->det[F64],
                                          op->links[F32], op->det[F32], op->links[F16S],
                                          op->links[BF16S]);
    CREATE_HIP(hipGetLastError());

    // 3. clover blocks (FP64) and their lower-precision copies
    dim3 gs((g.Vh + 127) / 128, 2);
    clover_kernel<<<gs, 128, 0, st>>>(g, su3, theta, m0, csw, (double2*)op->clover[F64]);
    CREATE_HIP(hipGetLastError());
    convert_site_reals<<<gs, 128, 0, st>>>(g, 72, (const double*)op->clover[F64],
                                           (float*)op->clover[F32], (_Float16*)op->clover[F16S],
                                           (uint16_t*)op->clover[BF16S]);
    CREATE_HIP(hipGetLastError());
    compact_clover_kernel<<<gs, 128, 0, st>>>(g, (const double2*)op->clover[F64],
                                              (double2*)op->clover54[F64], (float*)op->clover54[F32],
                                              (_Float16*)op->clover54[F16S],
                                              (uint16_t*)op->clover54[BF16S]);
    CREATE_HIP(hipGetLastError());
    // their inverses (the even-odd reduced operator divides by the odd-site blocks)
    clover_inv_kernel<<<gs, 128, 0, st>>>(g, (const double2*)op->clover[F64],
                                          (double2*)op->cloverinv[F64]);
    CREATE_HIP(hipGetLastError());
    convert_site_reals<<<gs, 128, 0, st>>>(g, 72, (const double*)op->cloverinv[F64],
                                           (float*)op->cloverinv[F32],
                                           (_Float16*)op->cloverinv[F16S],
                                           (uint16_t*)op->cloverinv[BF16S]);
    CREATE_HIP(hipGetLastError());
    CREATE_HIP(hipStreamSynchronize(st));
#undef CREATE_HIP
    *out = op;
    return QDW_OK;
}

extern "C" int qdw_destroy(qdw_op* op)
{
    if (!op) return QDW_OK;
    (void)hipDeviceSynchronize();
    delete op;  // the device and host blocks stay with the caller
    return QDW_OK;
}

extern "C" long qdw_volume(const qdw_op* op) { return op ? (long)op->g.V : 0; }

extern "C" size_t qdw_field_bytes(const qdw_op* op, qdw_prec prec)
{
    if (!op || prec < QDW_F64 || prec > QDW_BF16S) return 0;
    return spinor_bytes(op->g, prec);
}

extern "C" int qdw_pack(const qdw_op* op, const double* canonical, void* eo, qdw_prec prec,
                        void* stream)
{
    QDW_CHECK(op && canonical && eo, QDW_EINVAL, "qdw_pack: null argument");
    const Geom& g = op->g;
    dim3 gr((g.Vh + 255) / 256, 2);
    hipStream_t st = (hipStream_t)stream;
    switch (prec) {
    case QDW_F64: pack_kernel<F64><<<gr, 256, 0, st>>>(g, canonical, eo); break;
    case QDW_F32: pack_kernel<F32><<<gr, 256, 0, st>>>(g, canonical, eo); break;
    case QDW_F16S: pack_kernel<F16S><<<gr, 256, 0, st>>>(g, canonical, eo); break;
    case QDW_BF16S: pack_kernel<BF16S><<<gr, 256, 0, st>>>(g, canonical, eo); break;
    default: QDW_CHECK(false, QDW_EINVAL, "qdw_pack: bad precision");
    }
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}

extern "C" int qdw_unpack(const qdw_op* op, const void* eo, double* canonical, qdw_prec prec,
                          void* stream)
{
    QDW_CHECK(op && canonical && eo, QDW_EINVAL, "qdw_unpack: null argument");
    const Geom& g = op->g;
    dim3 gr((g.Vh + 255) / 256, 2);
    hipStream_t st = (hipStream_t)stream;
    switch (prec) {
    case QDW_F64: unpack_kernel<F64><<<gr, 256, 0, st>>>(g, eo, canonical); break;
    case QDW_F32: unpack_kernel<F32><<<gr, 256, 0, st>>>(g, eo, canonical); break;
    case QDW_F16S: unpack_kernel<F16S><<<gr, 256, 0, st>>>(g, eo, canonical); break;
    case QDW_BF16S: unpack_kernel<BF16S><<<gr, 256, 0, st>>>(g, eo, canonical); break;
    default: QDW_CHECK(false, QDW_EINVAL, "qdw_unpack: bad precision");
    }
    QDW_LAUNCH_CHECK();
    return QDW_OK;
}
