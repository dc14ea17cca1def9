// qdw_host.h -- host-side state of an operator and error plumbing of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/qdw.h"
#include "qdw_internal.h"

struct qdw_op {
    qdw::Geom g;
    double m0, csw;
    int device;
    // per precision (index = qdw::Prec): compressed links (rows 0, 1 of the U(3) link),
    // link determinants exp(3 i theta) (F64: one double each, see encode_phase; F32: float2
    // arrays; the 16-bit formats keep them inside the link chunks), clover blocks
    void* links[4];
    void* det[4];
    void* clover[4];
    void* cloverinv[4];    // per precision: inverses of the clover blocks (same format)
    void* clover54[4];     // per precision: the compact clover form the D kernels read
    void* full_links;      // optional, caller-owned: FP64 links as full 3x3 matrices
    // per precision: shape of the D kernel (sites per parity of a workgroup, time slices
    // per walk chunk, software-pipelined hop loop, walk order, marching form); other site
    // kernels use g
    struct { int ts, nt, pipe, walk, march; } dw_shape[4];
    // reduction scratch: per-workgroup partial sums and the final scalars
    double* partials;      // device, kMaxPartials * kMaxScalars doubles
    double* scalars;       // device, kMaxScalars doubles
    double* host_scalars;  // pinned host, kHostScalars doubles
};

namespace qdw {

constexpr int kMaxPartials = 2048;  // workgroups of a reduction launch
constexpr int kMaxScalars = 64;     // doubles produced by one fused reduction
constexpr int kHostScalars = 1024;  // doubles the host can read back in one copy
constexpr int kMaxRhs = 64;         // right-hand sides of one multi-right-hand-side launch

void set_error(const std::string& msg);

inline size_t spinor_bytes(const Geom& g, int prec)
{
    const size_t r = prec == F64 ? 8 : prec == F32 ? 4 : 2;
    return (size_t)2 * padded(g.Vh) * 24 * r;
}

}  // namespace qdw

#define QDW_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            qdw::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
            return QDW_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

#define QDW_CHECK(cond, code, msg)                                                     \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            qdw::set_error(msg);                                                       \
            return (code);                                                             \
        }                                                                              \
    } while (0)

#define QDW_LAUNCH_CHECK() QDW_HIP(hipGetLastError())
