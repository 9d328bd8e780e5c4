// Registry part: F32 fused-step configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f32_step(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {KL_ST_SET(float, KL_F32, 1), KL_ST_SET(float, KL_F32, 2), KL_ST_SET(float, KL_F32, 4)};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
