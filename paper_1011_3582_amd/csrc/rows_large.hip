// Row kernels (stage 2, collide, init/set, real transforms) for grid sizes: 768 1024 2048.
#include "launch_rows.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_ROWS(768)
FFTLB_INSTANTIATE_ROWS(1024)
FFTLB_INSTANTIATE_ROWS(2048)
}  // namespace fftlb
