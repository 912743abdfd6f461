// Column kernels (convection and derivative passes, every plan) for grid sizes: 2048.
#include "launch_cols.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_COLS(2048)
}  // namespace fftlb
