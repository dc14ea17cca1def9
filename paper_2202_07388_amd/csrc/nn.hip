// nn.hip -- learned gauge-covariant preconditioner (parallel-transport layers).
#include "blas.h"

namespace qdw {

size_t nn_precond_workspace(const qdw_op*) { return 0; }

int nn_precondition(qdw_op*, const void*, const void*, void*, double, char*, hipStream_t)
{
    QDW_CHECK(false, QDW_EINVAL, "the learned preconditioner is not available in this build");
}

}  // namespace qdw
