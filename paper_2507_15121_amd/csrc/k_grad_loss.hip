// Kernel instances: fused residual + MTTKRP gradient that also sums the loss.
#include "kernel_impl.h"

namespace amped {
namespace dev {

KernelFn pick_grad_loss(int nin, int lpr, bool scalar, bool buf) { return pick_any<float, 3>(nin, lpr, scalar, buf); }

}  // namespace dev
}  // namespace amped
