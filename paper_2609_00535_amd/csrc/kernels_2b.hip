// Kernel instances and launchers for 2-D, N = 8..12, 14, 16.
#include "kernels.hpp"

namespace slbm {
SLBM_LAUNCHER_SET(2b, SLBM_ORDERS_2B)
}  // namespace slbm
