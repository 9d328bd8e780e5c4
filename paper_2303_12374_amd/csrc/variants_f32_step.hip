// Registry part: F32 fused-step configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f32_step(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {KL_ST_SET(float, KL_F32, 1), KL_ST_SET(float, KL_F32, 2), KL_ST_SET(float, KL_F32, 4),
                                             KL_STW(float, KL_F32, 4, 4, 32, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(float, KL_F32, 4, 4, 64, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(float, KL_F32, 4, 4, 16, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(float, KL_F32, 4, 2, 32, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(float, KL_F32, 2, 4, 32, 2, 1, 1, FUSE_HALO3, "_h3"),
                                             KL_STW(float, KL_F32, 4, 4, 30, 2, 1, 1, FUSE_RING6 | FUSE_HALO3, "_r6h"),
                                             KL_STY(float, KL_F32, 4, 4, 16, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(float, KL_F32, 4, 4, 32, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(float, KL_F32, 4, 4, 64, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(float, KL_F32, 4, 8, 32, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(float, KL_F32, 4, 8, 16, 2, 1, FUSE_HALO3, "_h3y"),
                                             KL_STY(float, KL_F32, 4, 8, 64, 2, 1, FUSE_HALO3, "_h3y")};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
