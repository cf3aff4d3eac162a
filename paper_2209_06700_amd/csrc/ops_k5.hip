// Instantiation of the matrix-free operator kernels for degree 5.
#include "op_kernel.h"

namespace rk {
hipError_t launch_op_k5(const OpLaunch& L) { return dev::launch_op_k<5>(L); }
hipError_t launch_op_list_k5(const OpLaunch* L, int count, hipStream_t st) {
    return dev::launch_op_list_k<5>(L, count, st);
}
}  // namespace rk
