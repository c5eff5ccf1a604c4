// Kernels and launchers for probe side m = 128 (every plan variant, level count
// and finalize shape of that side).
#include "kernels.hpp"

namespace emg {
template struct Launchers<128>;
}  // namespace emg
