// assign_mfma.hip -- split-BF16 MFMA log-likelihood kernel (not yet built).
#include "dpmm_common.hpp"
#include "kernels.hpp"

namespace dpmm {

void launch_assign_bf16(const Ws&, const AssignArgs&, hipStream_t) {}

}  // namespace dpmm
