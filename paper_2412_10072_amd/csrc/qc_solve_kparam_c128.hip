// Solve kernels for param terms, complex128 data, FP64 arithmetic.
#include "qc_solve_kernels.h"

namespace qc {
template hipError_t launch_solve_kind<KIND_DELAY, double, double>(const SolveLaunch&, const SplitLaunch*, hipStream_t, size_t*);
}  // namespace qc
