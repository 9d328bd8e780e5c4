// Registry part: F64 configurations of the fused advec_u + diff_uvw pass.
#include "variants.hpp"

namespace kl {

void add_variants_f64_ad(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {
        Variant{"default", KL_KERNEL_ADVEC_DIFF, KL_F64, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                &launch_plain<double, KL_KERNEL_ADVEC_DIFF>, nullptr, nullptr},
        KL_AD_SET(double, KL_F64, 1), KL_AD_SET(double, KL_F64, 2),
        KL_ADW(double, KL_F64, 2, 8, 256, 2, 1, 1, FUSE_HALO3, "_h3"), KL_ADW(double, KL_F64, 2, 8, 64, 2, 1, 1, FUSE_HALO3, "_h3")};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
