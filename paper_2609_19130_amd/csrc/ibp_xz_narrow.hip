// The general x and z transforms for factorisations whose radices are all
// 2, 3, 4, 5 or 8: the kernels of ibp_xz_kernels.hpp without the radix-7 and
// radix-11 butterflies, the direct-sum stage and Bluestein's convolution.
// Those stages set a kernel's register count even when a plan never runs
// them (FP64 LDS transform: 165 VGPRs, 3 waves per SIMD, against 92 without).
#include "ibp_xz_kernels.hpp"

namespace ibp {

IBP_XZ_FAMILY(, false)

}  // namespace ibp
