// Generated instantiations of the fused OMP kernel (see omp_kernel.h).
#include "omp_kernel.h"

namespace smdl_omp {
template hipError_t launch_one<4, 12, 16, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 8, 16, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<12, 8, 16, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 8, 16, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<4, 8, 32, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 8, 32, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 8, 32, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 16, 32, 4>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<4, 16, 64, 2>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<8, 16, 64, 1>(const OmpArgs&, int, int, hipStream_t);
template hipError_t launch_one<16, 16, 64, 2>(const OmpArgs&, int, int, hipStream_t);
}  // namespace smdl_omp
