// Instantiation of the matrix-free operator kernels for degree 3.
#include "op_kernel.h"

namespace rk {
hipError_t launch_op_k3(const OpLaunch& L) { return dev::launch_op_k<3>(L); }
hipError_t launch_op_list_k3(const OpLaunch* L, int count, hipStream_t st) {
    return dev::launch_op_list_k<3>(L, count, st);
}
}  // namespace rk
