// Registry part: F64 fused-step configurations.
#include "variants.hpp"

namespace kl {

void add_variants_f64_step(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {KL_ST_SET(double, KL_F64, 1), KL_ST_SET(double, KL_F64, 2)};
    out.insert(out.end(), v.begin(), v.end());
}

}  // namespace kl
