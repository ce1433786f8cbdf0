// Kernel instances and launchers for 2-D, N = 2..7.
#include "kernels.hpp"

namespace slbm {
SLBM_LAUNCHER_SET(2a, SLBM_ORDERS_2A)
}  // namespace slbm
