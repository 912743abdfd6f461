// Row kernels (stage 2, collide, init/set, real transforms) for grid sizes: 256 384 512.
#include "launch_rows.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_ROWS(256)
FFTLB_INSTANTIATE_ROWS(384)
FFTLB_INSTANTIATE_ROWS(512)
}  // namespace fftlb
