// Column kernels (convection and derivative passes, every plan) for grid sizes: 4 8 16 32 48 64.
#include "launch_cols.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_COLS(4)
FFTLB_INSTANTIATE_COLS(8)
FFTLB_INSTANTIATE_COLS(16)
FFTLB_INSTANTIATE_COLS(32)
FFTLB_INSTANTIATE_COLS(48)
FFTLB_INSTANTIATE_COLS(64)
}  // namespace fftlb
