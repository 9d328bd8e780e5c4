// Registry of F64 tendency-kernel configurations (index 0: the default).
#include "variants.hpp"

namespace kl {

void add_variants_f64_zc(int kernel, std::vector<Variant> &out);
void add_variants_f64_zl1(int kernel, std::vector<Variant> &out);
void add_variants_f64_zl2(int kernel, std::vector<Variant> &out);
void add_variants_f64_x(int kernel, std::vector<Variant> &out);
void add_variants_f64_nt(int kernel, std::vector<Variant> &out);
void add_variants_f64_step(std::vector<Variant> &out);
void add_variants_f64_small(int kernel, std::vector<Variant> &out);
void add_variants_f64_rev(int kernel, std::vector<Variant> &out);
void add_variants_f64_les(int kernel, std::vector<Variant> &out);
void add_variants_f64_split(std::vector<Variant> &out);
void add_variants_f64_ad(std::vector<Variant> &out);

static std::vector<Variant> build_f64(int kernel)
{
    std::vector<Variant> v;
    if (kernel == KL_KERNEL_STEP) {  // index 0: a fused step with scalar lanes (fits any itot)
        add_variants_f64_step(v);
        return v;
    }
    if (kernel == KL_KERNEL_ADVEC_DIFF) {
        add_variants_f64_ad(v);
        return v;
    }
    if (kernel == KL_KERNEL_ADVEC_U_2I5 || kernel == KL_KERNEL_DIFF_SMAG) {
        v.push_back(Variant{"default", kernel, KL_F64, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                            kernel == KL_KERNEL_ADVEC_U_2I5 ? &launch_plain<double, KL_KERNEL_ADVEC_U_2I5>
                                                            : &launch_plain<double, KL_KERNEL_DIFF_SMAG>,
                            nullptr, nullptr});
        add_variants_f64_les(kernel, v);
        return v;
    }
    v.push_back(Variant{"default", kernel, KL_F64, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                        kernel == KL_KERNEL_ADVEC_U ? &launch_plain<double, KL_KERNEL_ADVEC_U>
                                                    : &launch_plain<double, KL_KERNEL_DIFF_UVW>,
                        nullptr, nullptr});
        add_variants_f64_zc(kernel, v);
        add_variants_f64_zl1(kernel, v);
        add_variants_f64_zl2(kernel, v);
        add_variants_f64_x(kernel, v);
        add_variants_f64_nt(kernel, v);
        add_variants_f64_small(kernel, v);
        add_variants_f64_rev(kernel, v);
        if (kernel == KL_KERNEL_DIFF_UVW) add_variants_f64_split(v);
    return v;
}

const std::vector<Variant> &variants_f64(int kernel)
{
    static const std::vector<Variant> advec = build_f64(KL_KERNEL_ADVEC_U);
    static const std::vector<Variant> diff = build_f64(KL_KERNEL_DIFF_UVW);
    static const std::vector<Variant> step = build_f64(KL_KERNEL_STEP);
    static const std::vector<Variant> advec5 = build_f64(KL_KERNEL_ADVEC_U_2I5);
    static const std::vector<Variant> smag = build_f64(KL_KERNEL_DIFF_SMAG);
    static const std::vector<Variant> ad = build_f64(KL_KERNEL_ADVEC_DIFF);
    switch (kernel) {
    case KL_KERNEL_ADVEC_U: return advec;
    case KL_KERNEL_DIFF_UVW: return diff;
    case KL_KERNEL_STEP: return step;
    case KL_KERNEL_ADVEC_U_2I5: return advec5;
    case KL_KERNEL_ADVEC_DIFF: return ad;
    default: return smag;
    }
}

}  // namespace kl
