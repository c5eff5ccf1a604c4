// Kernels and launchers for probe side m = 32 (every plan variant, level count
// and finalize shape of that side).
#include "kernels.hpp"

namespace emg {
template struct Launchers<32>;
}  // namespace emg
