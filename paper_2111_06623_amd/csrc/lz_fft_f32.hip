// FFT kernels of the Liouvillian application, single precision.
#include "lz_fft_kernels.h"

namespace lz {
template struct LaunchFft<float>;
template hipError_t enable_large_lds_fft<float>();
}  // namespace lz
