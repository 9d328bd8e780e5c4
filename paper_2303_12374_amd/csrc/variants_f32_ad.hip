// Registry part: F32 configurations of the fused advec_u + diff_uvw pass.
#include "variants.hpp"

namespace kl {

void add_variants_f32_ad(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {
        Variant{"default", KL_KERNEL_ADVEC_DIFF, KL_F32, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                &launch_plain<float, KL_KERNEL_ADVEC_DIFF>, nullptr, nullptr},
        KL_AD_SET(float, KL_F32, 1), KL_AD(float, KL_F32, 1, 16, 64, 2, 1), KL_AD_SET(float, KL_F32, 2), KL_AD_SET(float, KL_F32, 4),
        KL_ADW(float, KL_F32, 4, 8, 256, 2, 1, 1, FUSE_HALO3, "_h3"), KL_ADW(float, KL_F32, 4, 8, 128, 2, 1, 1, FUSE_HALO3, "_h3")};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
