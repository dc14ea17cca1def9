// blas.hip -- second reduction pass and its scalar programs.
#include "blas.h"

namespace qdw {

// One workgroup sums the per-workgroup partials and runs the scalar program `op`.
__global__ __launch_bounds__(256) void finalize_kernel(const double* partials, int nblk, int ns,
                                                       double* out, int op, int k)
{
    finalize_body(partials, nblk, ns, out, op, k);
}

}  // namespace qdw

// ---------------------------------------------------------------- C ABI

namespace {

template <int P>
struct Dot {
    static constexpr int NS = 2;
    const void* x;
    const void* y;
    int Vh;
    __device__ void operator()(const qdw::Unit& u, double* acc) const
    {
        qdw::cx<double> a[4], b[4];
        qdw::ld4<P, double>(x, Vh, u.par, u.g, u.i, a);
        qdw::ld4<P, double>(y, Vh, u.par, u.g, u.i, b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const qdw::cx<double> z = qdw::cmul_conj(a[k], b[k]);
            acc[0] += z.re;
            acc[1] += z.im;
        }
    }
};

template <template <int> class F, class Fill>
int by_prec(qdw_prec prec, Fill fill)
{
    switch (prec) {
    case QDW_F64: { F<qdw::F64> f; return fill(f); }
    case QDW_F32: { F<qdw::F32> f; return fill(f); }
    case QDW_F16S: { F<qdw::F16S> f; return fill(f); }
    case QDW_BF16S: { F<qdw::BF16S> f; return fill(f); }
    default: QDW_CHECK(false, QDW_EINVAL, "bad precision");
    }
}

template <int P> using AxpbySame = qdw::Axpby<P, P>;

}  // namespace

extern "C" int qdw_axpby(qdw_op* op, double a, const void* x, double b, void* y, qdw_prec prec,
                         void* stream)
{
    QDW_CHECK(op && x && y, QDW_EINVAL, "qdw_axpby: null argument");
    hipStream_t st = (hipStream_t)stream;
    return by_prec<AxpbySame>(prec, [&](auto& f) {
        f.x = x; f.y = y; f.a = a; f.b = b; f.Vh = op->g.Vh;
        return qdw::run_map(op, f, st);
    });
}

extern "C" int qdw_norm2(qdw_op* op, const void* x, qdw_prec prec, double* out, void* stream)
{
    QDW_CHECK(op && x && out, QDW_EINVAL, "qdw_norm2: null argument");
    hipStream_t st = (hipStream_t)stream;
    int rc = by_prec<qdw::Norm2>(prec, [&](auto& f) {
        f.x = x; f.Vh = op->g.Vh;
        return qdw::run_map(op, f, st, op->scalars + qdw::S_TMP);
    });
    if (rc) return rc;
    return qdw::read_scalars(op, qdw::S_TMP, 1, out, st);
}

extern "C" int qdw_cdot(qdw_op* op, const void* x, const void* y, qdw_prec prec, double* out,
                        void* stream)
{
    QDW_CHECK(op && x && y && out, QDW_EINVAL, "qdw_cdot: null argument");
    hipStream_t st = (hipStream_t)stream;
    int rc = by_prec<Dot>(prec, [&](auto& f) {
        f.x = x; f.y = y; f.Vh = op->g.Vh;
        return qdw::run_map(op, f, st, op->scalars + qdw::S_TMP);
    });
    if (rc) return rc;
    return qdw::read_scalars(op, qdw::S_TMP, 2, out, st);
}

namespace {

template <int PX>
int convert_to(qdw_op* op, const void* x, void* y, qdw_prec py, double s, hipStream_t st)
{
    const int Vh = op->g.Vh;
    switch (py) {
    case QDW_F64: return qdw::run_map(op, qdw::Axpby<PX, qdw::F64>{x, y, s, 0.0, Vh}, st);
    case QDW_F32: return qdw::run_map(op, qdw::Axpby<PX, qdw::F32>{x, y, s, 0.0, Vh}, st);
    case QDW_F16S: return qdw::run_map(op, qdw::Axpby<PX, qdw::F16S>{x, y, s, 0.0, Vh}, st);
    case QDW_BF16S: return qdw::run_map(op, qdw::Axpby<PX, qdw::BF16S>{x, y, s, 0.0, Vh}, st);
    default: QDW_CHECK(false, QDW_EINVAL, "qdw_convert: bad precision");
    }
}

}  // namespace

extern "C" int qdw_convert(qdw_op* op, const void* x, qdw_prec px, void* y, qdw_prec py,
                           double s, void* stream)
{
    QDW_CHECK(op && x && y, QDW_EINVAL, "qdw_convert: null argument");
    QDW_CHECK(x != y, QDW_EINVAL, "qdw_convert: x and y must be distinct");
    hipStream_t st = (hipStream_t)stream;
    switch (px) {
    case QDW_F64: return convert_to<qdw::F64>(op, x, y, py, s, st);
    case QDW_F32: return convert_to<qdw::F32>(op, x, y, py, s, st);
    case QDW_F16S: return convert_to<qdw::F16S>(op, x, y, py, s, st);
    case QDW_BF16S: return convert_to<qdw::BF16S>(op, x, y, py, s, st);
    default: QDW_CHECK(false, QDW_EINVAL, "qdw_convert: bad precision");
    }
}
