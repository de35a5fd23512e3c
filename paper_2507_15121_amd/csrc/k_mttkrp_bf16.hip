// Kernel instances: MTTKRP with bfloat16 factors.
#include "kernel_impl.h"

namespace amped {
namespace dev {

// Rows of up to 64 bytes (rank <= 32) use 8 bytes per lane, so a wave still
// covers 8 rows per gather at rank 32 (16-byte lanes would make 16 narrow
// groups); longer rows use 16 bytes per lane.  lpr counts 16-byte lanes.
#ifndef AMPED_BF16_NARROW
#define AMPED_BF16_NARROW 1
#endif
template <int NIN, typename T, int KIND, bool BUF>
KernelFn pick_vec(int lpr)
{
    constexpr int RPL = 16 / sizeof(T);
    if constexpr (NIN > kMaxVecNin) {
        return nullptr;
    } else {
        if (AMPED_BF16_NARROW && lpr <= 4) {
            switch (lpr) {
            case 2: return mttkrp_kernel<NIN, 4, 4, T, KIND, BUF>;
            case 4: return mttkrp_kernel<NIN, 8, 4, T, KIND, BUF>;
            default: return nullptr;
            }
        }
        switch (lpr) {
        case 4: return mttkrp_kernel<NIN, 4, RPL, T, KIND, BUF>;
        case 8: return mttkrp_kernel<NIN, 8, RPL, T, KIND, BUF>;
        case 16: return mttkrp_kernel<NIN, 16, RPL, T, KIND, BUF>;
        case 32:
            if constexpr (std::is_same<T, float>::value) return mttkrp_kernel<NIN, 32, RPL, T, KIND, BUF>;
            else return nullptr;
        default: return nullptr;
        }
    }
}

template <int NIN, typename T, int KIND>
KernelFn pick_nin(int lpr, bool scalar, bool buf)
{
    if (scalar) return mttkrp_kernel<NIN, 64, 1, T, KIND, false>;
    return buf ? pick_vec<NIN, T, KIND, true>(lpr) : pick_vec<NIN, T, KIND, false>(lpr);
}

template <typename T, int KIND>
KernelFn pick_any(int nin, int lpr, bool scalar, bool buf)
{
    switch (nin) {
    case 1: return pick_nin<1, T, KIND>(lpr, scalar, buf);
    case 2: return pick_nin<2, T, KIND>(lpr, scalar, buf);
    case 3: return pick_nin<3, T, KIND>(lpr, scalar, buf);
    case 4: return pick_nin<4, T, KIND>(lpr, scalar, buf);
    case 5: return pick_nin<5, T, KIND>(lpr, scalar, buf);
    case 6: return pick_nin<6, T, KIND>(lpr, scalar, buf);
    case 7: return pick_nin<7, T, KIND>(lpr, scalar, buf);
    default: return nullptr;
    }
}

KernelFn pick_mttkrp_bf16(int nin, int lpr, bool scalar, bool buf)
{
    return pick_any<uint16_t, 0>(nin, lpr, scalar, buf);
}

}  // namespace dev
}  // namespace amped
