// Solve kernels for diag terms, complex64 data, FP32 products and compensated sums.
#include "qc_solve_kernels.h"

namespace qc {
template hipError_t launch_solve_kind<KIND_DIAG, float, float>(const SolveLaunch&, const SplitLaunch*, hipStream_t, size_t*);
}  // namespace qc
