// Generated instantiations of the fused OMP kernel (see omp_kernel.h).
#include "omp_kernel.h"

namespace smdl_omp {
template hipError_t launch_one<4, 16, 16, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 12, 16, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<12, 12, 16, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 12, 16, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<4, 12, 32, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 12, 32, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 12, 32, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<4, 8, 64, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 8, 64, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 8, 64, 1>(const OmpArgs&, int, int, hipStream_t);
}  // namespace smdl_omp
