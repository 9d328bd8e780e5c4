// Registry part: F32 top-down slab order configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f32_rev(int kernel, std::vector<Variant> &out)
{
#define KL_LIST(KERN) {KL_REV_SET(float, KL_F32, KERN, 2), KL_REV_SET(float, KL_F32, KERN, 4), KL_OCC_SET(float, KL_F32, KERN, 4)}
    static const std::vector<Variant> advec = KL_LIST(KL_KERNEL_ADVEC_U);
    static const std::vector<Variant> diff = KL_LIST(KL_KERNEL_DIFF_UVW);
#undef KL_LIST
    const auto &v = kernel == KL_KERNEL_ADVEC_U ? advec : diff;
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
