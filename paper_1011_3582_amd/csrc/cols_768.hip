// Column kernels (convection and derivative passes, every plan) for grid sizes: 768 1024.
#include "launch_cols.hpp"

namespace fftlb {
FFTLB_INSTANTIATE_COLS(768)
FFTLB_INSTANTIATE_COLS(1024)
}  // namespace fftlb
