// Kernels and launchers for probe side m = 64 (every plan variant, level count
// and finalize shape of that side).
#include "kernels.hpp"

namespace emg {
template struct Launchers<64>;
}  // namespace emg
