// blas.hip -- second reduction pass and its scalar programs.
#include "blas.h"

namespace qdw {

// One workgroup sums the per-workgroup partials in a fixed order (strided per lane,
// then a fixed tree), then runs the scalar program `op`.
__global__ __launch_bounds__(256) void finalize_kernel(const double* partials, int nblk, int ns,
                                                       double* out, int op, int k)
{
    __shared__ double red[256];
    __shared__ double sums[kMaxScalars];
    for (int j = 0; j < ns; ++j) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) s += partials[(long)b * ns + j];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
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

}  // namespace qdw
