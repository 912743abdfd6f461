// Column kernels (convection and derivative passes, every plan) for grid sizes: 384 512.
#include "launch_cols.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_COLS(384)
FFTLB_INSTANTIATE_COLS(512)
}  // namespace fftlb
