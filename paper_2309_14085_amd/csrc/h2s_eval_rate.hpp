// h2s_eval_rate.hpp -- launcher of the register-resident kernel-evaluation
// rate loop (h2s_eval_rate.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2s {

// Evaluations one launch of `blocks` blocks and `passes` passes performs, and
// the doubles it writes to `out` (one per thread).
int64_t eval_rate_evals(int blocks, int passes);
int64_t eval_rate_outputs(int blocks);

// One launch: kernel kind, dimension d, float or double arithmetic, the
// kernel-function table `tab` (device; the product's table for this kind) and
// scalar parameters (kparam = -1/h^2 for the Gaussian; kc as the product).
hipError_t launch_eval_rate(int kind, int d, bool fp32, int blocks, const double *tab, double kparam,
                            const double kc[3], int passes, double *out, hipStream_t s);

} // namespace h2s
