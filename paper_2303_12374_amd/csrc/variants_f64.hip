// Registry of FP64 tendency-kernel configurations.
#include "variants.hpp"

namespace kl {

const std::vector<Variant> &variants_f64(int kernel)
{
#define KL_LIST(KERN)                                                                         \
    {Variant{"default", KERN, KL_F64, FAMILY_PLAIN, 1, 256, 1, 1, 0, &launch_plain<double, KERN>, nullptr, nullptr}, \
     KL_ZC_BLOCKS(double, KL_F64, KERN, 1), KL_ZC_BLOCKS(double, KL_F64, KERN, 2), KL_ZL_BLOCKS(double, KL_F64, KERN, 1), KL_ZL_BLOCKS(double, KL_F64, KERN, 2) \
    }
    static const std::vector<Variant> advec = KL_LIST(KL_KERNEL_ADVEC_U);
    static const std::vector<Variant> diff = KL_LIST(KL_KERNEL_DIFF_UVW);
#undef KL_LIST
    return kernel == KL_KERNEL_ADVEC_U ? advec : diff;
}

}  // namespace kl
