// Column kernels (convection and derivative passes, every plan) for grid sizes: 96 128 192 256.
#include "launch_cols.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_COLS(96)
FFTLB_INSTANTIATE_COLS(128)
FFTLB_INSTANTIATE_COLS(192)
FFTLB_INSTANTIATE_COLS(256)
}  // namespace fftlb
