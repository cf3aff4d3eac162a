// Instantiation of the matrix-free operator kernels for degree 4.
#include "op_kernel.h"

namespace rk {
hipError_t launch_op_k4(const OpLaunch& L) { return dev::launch_op_k<4>(L); }
hipError_t launch_op_list_k4(const OpLaunch* L, int count, hipStream_t st) {
    return dev::launch_op_list_k<4>(L, count, st);
}
}  // namespace rk
