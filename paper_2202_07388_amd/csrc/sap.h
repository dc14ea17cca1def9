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

enum { S_SAP = 12 };  // scalar slot used by the preconditioner's scaling pass

int make_block_geom(const Geom& g, const int bs[4], BlockGeom* B);

size_t sap_workspace(const qdw_op* op, int sdtype);

// phi = M_SAP rho (FP64 fields); |rho| must be passed in (it sets the storage scale)
int sap_run(qdw_op* op, const void* rho, void* phi, double rho_norm, int ncy, int nmr,
            const BlockGeom& B, int sdtype, char* work, hipStream_t st);

// ncy Schwarz cycles on the storage-precision fields rs (residual, updated), psis
// (solution, accumulated) and delta (scratch), for nrhs right-hand sides at bat's stride
int sap_cycles(qdw_op* op, const BlockGeom& B, int sdtype, int ncy, int nmr, void* rs,
               void* psis, void* delta, const RhsStride& bat, int nrhs, hipStream_t st);

}  // namespace qdw
