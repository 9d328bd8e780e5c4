// Registry part: F64 configurations of advec_u_2i5 and diff_smag.
#include "variants.hpp"

namespace kl {

void add_variants_f64_split(std::vector<Variant> &out)
{
    static const std::vector<Variant> v = {
        KL_ZL3(double, KL_F64, 2, 4, 128, 2, 1),
        KL_ZL3(double, KL_F64, 2, 4, 256, 3, 1),
        KL_ZL3(double, KL_F64, 2, 8, 64, 2, 1),
        KL_ZL3(double, KL_F64, 2, 4, 64, 2, 1),
        KL_ZL3(double, KL_F64, 2, 8, 256, 3, 1),
        KL_ZL3(double, KL_F64, 2, 8, 128, 3, 1),
        KL_ZL3(double, KL_F64, 2, 16, 128, 3, 1),
        KL_ZL3(double, KL_F64, 2, 16, 64, 2, 1)};
    out.insert(out.end(), v.begin(), v.end());
}

void add_variants_f64_les(int kernel, std::vector<Variant> &out)
{
    if (kernel == KL_KERNEL_ADVEC_U_2I5) {
        static const std::vector<Variant> v = {
        KL_A5P(double, KL_F64, 2, 8, 64, 2, 1),
        KL_A5R(double, KL_F64, 2, 4, 64, 2, 1),
        KL_A5R(double, KL_F64, 2, 4, 128, 2, 1),
        KL_A5R(double, KL_F64, 2, 8, 64, 2, 1),
        KL_A5R(double, KL_F64, 1, 8, 64, 2, 1),
        KL_A5R(double, KL_F64, 2, 8, 128, 2, 1),
        KL_A5RH(double, KL_F64, 2, 8, 128, 2, 1, 5),
        KL_A5RH(double, KL_F64, 2, 8, 64, 2, 1, 5),
        KL_A5RH(double, KL_F64, 2, 8, 128, 2, 1, 3),
        KL_A5R(double, KL_F64, 1, 16, 64, 2, 1),
        KL_A5S(double, KL_F64, 2, 8, 64, 2, 1),
        KL_A5S(double, KL_F64, 2, 4, 64, 2, 1),
        KL_A5P(double, KL_F64, 1, 8, 64, 2, 1),
        KL_A5P(double, KL_F64, 1, 16, 64, 2, 1),
        KL_A5P(double, KL_F64, 2, 4, 64, 2, 1),
        KL_A5(double, KL_F64, 2, 4, 64, 2, 1),
        KL_A5(double, KL_F64, 2, 8, 64, 2, 1),
        KL_A5(double, KL_F64, 2, 4, 128, 2, 1),
        KL_A5(double, KL_F64, 1, 8, 64, 2, 1),
        KL_A5(double, KL_F64, 1, 16, 64, 2, 1),
        KL_A5(double, KL_F64, 2, 2, 64, 2, 1),
        KL_A5(double, KL_F64, 2, 4, 32, 0, 0),
        KL_A5(double, KL_F64, 1, 8, 16, 0, 0),
        KL_A5(double, KL_F64, 2, 4, 256, 3, 1)};
        out.insert(out.end(), v.begin(), v.end());
    } else if (kernel == KL_KERNEL_DIFF_SMAG) {
        static const std::vector<Variant> v = {
        KL_S2(double, KL_F64, 1, 8, 64, 2, 1),
        KL_S2(double, KL_F64, 1, 4, 64, 2, 1),
        KL_S2(double, KL_F64, 2, 4, 64, 2, 1),
        KL_S2(double, KL_F64, 1, 8, 32, 0, 0),
        KL_S2(double, KL_F64, 2, 2, 64, 2, 1),
        KL_S2(double, KL_F64, 1, 16, 64, 2, 1),
        KL_S2(double, KL_F64, 1, 8, 16, 0, 0),
        KL_S2(double, KL_F64, 2, 8, 64, 2, 1),
        KL_S2(double, KL_F64, 2, 8, 128, 2, 1),
        KL_S2R(double, KL_F64, 1, 8, 64, 2, 1)};
        out.insert(out.end(), v.begin(), v.end());
    }
}

}  // namespace kl
