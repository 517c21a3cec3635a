// Sweep kernels for one lattice (see msd_kernels.h); one translation unit per
// lattice keeps the template instantiations of the build parallel.
#include "msd_kernels.h"

namespace msd {
template hipError_t dispatch<8>(Op, const LaunchArgs&);
}  // namespace msd
