// Kernel instances: MTTKRP with bfloat16 factors.
#include "kernel_impl.h"

namespace amped {
namespace dev {

KernelFn pick_mttkrp_bf16(int nin, int lpr, bool scalar, bool buf)
{
    return pick_any<uint16_t, 0>(nin, lpr, scalar, buf);
}

}  // namespace dev
}  // namespace amped
