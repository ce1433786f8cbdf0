// Kernel instances and launchers for 3-D D3Q19, N = 2..6.
#include "kernels.hpp"

namespace slbm {
SLBM_LAUNCHER_SET(3d, SLBM_ORDERS_3D)
}  // namespace slbm
