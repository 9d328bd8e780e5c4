// Registry of FP32 tendency-kernel configurations.
#include "variants.hpp"

namespace kl {

const std::vector<Variant> &variants_f32(int kernel)
{
#define KL_LIST(KERN)                                                                       \
    {Variant{"default", KERN, KL_F32, FAMILY_PLAIN, 1, 256, 1, 1, 0, &launch_plain<float, KERN>, nullptr, nullptr}, \
     KL_ZC_BLOCKS(float, KL_F32, KERN, 1), KL_ZC_BLOCKS(float, KL_F32, KERN, 2),            \
     KL_ZC_BLOCKS(float, KL_F32, KERN, 4), KL_ZL_BLOCKS(float, KL_F32, KERN, 1), KL_ZL_BLOCKS(float, KL_F32, KERN, 2), KL_ZL_BLOCKS(float, KL_F32, KERN, 4) \
    }
    static const std::vector<Variant> advec = KL_LIST(KL_KERNEL_ADVEC_U);
    static const std::vector<Variant> diff = KL_LIST(KL_KERNEL_DIFF_UVW);
#undef KL_LIST
    return kernel == KL_KERNEL_ADVEC_U ? advec : diff;
}

}  // namespace kl
