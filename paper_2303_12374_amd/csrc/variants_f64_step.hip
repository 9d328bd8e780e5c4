// Registry part: F64 fused-step configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f64_step(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {KL_ST_SET(double, KL_F64, 1), KL_ST_SET(double, KL_F64, 2),
                                             KL_STW(double, KL_F64, 2, 4, 64, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(double, KL_F64, 2, 4, 32, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STY(double, KL_F64, 2, 4, 32, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(double, KL_F64, 2, 4, 64, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(double, KL_F64, 2, 8, 32, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(double, KL_F64, 2, 8, 64, 2, 1, FUSE_HALO3, "_h3y")};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
