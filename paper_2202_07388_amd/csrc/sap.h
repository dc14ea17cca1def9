// sap.h -- block geometry and the SAP preconditioner entry used by the GCR solver.
#pragma once

#include <cmath>

#include "blas.h"

namespace qdw {

struct BlockGeom {
    int bs[4];       // block extents (T, L1, L2, L3 order)
    int nb[4];       // blocks per direction (even, >= 2)
    int bvol;        // sites per block = workgroup size (64..256, whole wavefronts)
    int lstride[4];  // strides of the local site index (x3 fastest)
    int nblk;        // number of blocks
};

enum { S_SAP = 12, S_SAP_NEW = 13 };  // scalar slots of the preconditioner

// adaptive MR exits of the block solver (Sec. 3.2): on = 0 runs nmr steps always
struct SapAdapt {
    float alpha = 0.f;     // exit (1): |r_b| > alpha * previous, after >= 4 steps
    float tol = 0.f;       // exit (3): |r_b| < tol (in the units of the stored residual)
    int* steps = nullptr;  // optional: MR steps taken, one int per block of the colour
    int on = 0;
};

int make_block_geom(const Geom& g, const int bs[4], BlockGeom* B);

size_t sap_workspace(const qdw_op* op, int sdtype);

// phi = M_SAP rho (FP64 fields); |rho| must be passed in (it sets the storage scale);
// eo: block solves through the block's even-odd reduction
int sap_run(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy, int nmr,
            const BlockGeom& B, int sdtype, char* work, hipStream_t st, bool eo = false);

// adaptive SAP (Sec. 3.2): at most ncy_max cycles (stop when a cycle did not lower |r|), at
// most nmr_max MR steps per block with the exits of SapAdapt; tol is the absolute block
// tolerance for rho's scale; steps (device, optional) receives the per-block MR step counts,
// [cycle][colour][block of the colour]. The workspace's control ints (sap_ctrl) count the
// cycles; the third counts over all applications since sap_ctrl_reset_total.
int sap_adaptive_run(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy_max,
                     int nmr_max, double alpha, double tol, const BlockGeom& B, int sdtype,
                     char* work, int* steps, hipStream_t st);
int* sap_ctrl(const qdw_op* op, int sdtype, char* work);
int sap_ctrl_reset_total(int* ctrl, hipStream_t st);

// ncy Schwarz cycles on the storage-precision fields rs (residual, updated), psis
// (solution, accumulated) and delta (scratch), for nrhs right-hand sides at bat's stride
int sap_cycles(qdw_op* op, const BlockGeom& B, int sdtype, int ncy, int nmr, void* rs,
               void* psis, void* delta, const RhsStride& bat, int nrhs, hipStream_t st,
               bool eo = false);

}  // namespace qdw
