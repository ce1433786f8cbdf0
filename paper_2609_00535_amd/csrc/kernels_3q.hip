// Kernel instances and launchers for 3-D D3Q13, N = 2..6.
#include "kernels.hpp"

namespace slbm {
SLBM_LAUNCHER_SET(3q, SLBM_ORDERS_3Q)
}  // namespace slbm
