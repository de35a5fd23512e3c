// Kernel instances: sparse CP loss.
#include "kernel_impl.h"

namespace amped {
namespace dev {

KernelFn pick_loss(int nin, int lpr, bool scalar, bool buf) { return pick_any<float, 2>(nin, lpr, scalar, buf); }

}  // namespace dev
}  // namespace amped
