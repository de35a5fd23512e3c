// Kernel instances: fp32 MTTKRP.
#include "kernel_impl.h"

namespace amped {
namespace dev {

KernelFn pick_mttkrp_f32(int nin, int lpr, bool scalar, bool buf) { return pick_any<float, 0>(nin, lpr, scalar, buf); }

}  // namespace dev
}  // namespace amped
