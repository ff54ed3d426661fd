// Solve kernels for c2x2 terms, complex64 data, FP64 arithmetic.
#include "qc_solve_kernels.h"

namespace qc {
template hipError_t launch_solve_kind<KIND_C2X2, float, double>(const SolveLaunch&, const SplitLaunch*, hipStream_t, size_t*);
}  // namespace qc
