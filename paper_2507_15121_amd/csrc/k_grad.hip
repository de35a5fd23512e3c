// Kernel instances: fused residual + MTTKRP gradient.
#include "kernel_impl.h"

namespace amped {
namespace dev {

KernelFn pick_grad(int nin, int lpr, bool scalar, bool buf) { return pick_any<float, 1>(nin, lpr, scalar, buf); }

}  // namespace dev
}  // namespace amped
