// FFT kernels of the Liouvillian application, double precision.
#include "lz_fft_kernels.h"

namespace lz {
template struct LaunchFft<double>;
template hipError_t enable_large_lds_fft<double>();
}  // namespace lz
