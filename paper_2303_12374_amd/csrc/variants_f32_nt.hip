// Registry part: F32 streaming-field configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f32_nt(int kernel, std::vector<Variant> &out)
{
#define KL_LIST(KERN) {KL_NT2_SET(float, KL_F32, KERN, 2), KL_NT2_SET(float, KL_F32, KERN, 4)}
    // taller tiles (16 rows: fewer y-halo rows per row computed)
    static const std::vector<Variant> advec = [] {
        std::vector<Variant> l = KL_LIST(KL_KERNEL_ADVEC_U);
        const std::vector<Variant> t = {KL_ZLX(float, KL_F32, KL_KERNEL_ADVEC_U, 4, 16, 128, 2, 1, 1),
                                        KL_ZLX(float, KL_F32, KL_KERNEL_ADVEC_U, 4, 16, 128, 3, 1, 1),
                                        KL_ZLX(float, KL_F32, KL_KERNEL_ADVEC_U, 4, 16, 256, 3, 1, 1),
                                        KL_ZLX(float, KL_F32, KL_KERNEL_ADVEC_U, 4, 16, 32, 2, 1, 1)};
        l.insert(l.end(), t.begin(), t.end());
        return l;
    }();
    static const std::vector<Variant> diff = KL_LIST(KL_KERNEL_DIFF_UVW);
#undef KL_LIST
    const auto &v = kernel == KL_KERNEL_ADVEC_U ? advec : diff;
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
