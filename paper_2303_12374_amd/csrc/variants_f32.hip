// Registry of F32 tendency-kernel configurations (index 0: the default).
#include "variants.hpp"

namespace kl {

void add_variants_f32_zc(int kernel, std::vector<Variant> &out);
void add_variants_f32_zl1(int kernel, std::vector<Variant> &out);
void add_variants_f32_zl2(int kernel, std::vector<Variant> &out);
void add_variants_f32_zl4(int kernel, std::vector<Variant> &out);
void add_variants_f32_x(int kernel, std::vector<Variant> &out);
void add_variants_f32_nt(int kernel, std::vector<Variant> &out);
void add_variants_f32_step(std::vector<Variant> &out);
void add_variants_f32_small(int kernel, std::vector<Variant> &out);
void add_variants_f32_rev(int kernel, std::vector<Variant> &out);
void add_variants_f32_les(int kernel, std::vector<Variant> &out);
void add_variants_f32_split(std::vector<Variant> &out);
void add_variants_f32_ad(std::vector<Variant> &out);

static std::vector<Variant> build_f32(int kernel)
{
    std::vector<Variant> v;
    if (kernel == KL_KERNEL_STEP) {  // index 0: a fused step with scalar lanes (fits any itot)
        add_variants_f32_step(v);
        return v;
    }
    if (kernel == KL_KERNEL_ADVEC_DIFF) {
        add_variants_f32_ad(v);
        return v;
    }
    if (kernel == KL_KERNEL_ADVEC_U_2I5 || kernel == KL_KERNEL_DIFF_SMAG) {
        v.push_back(Variant{"default", kernel, KL_F32, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                            kernel == KL_KERNEL_ADVEC_U_2I5 ? &launch_plain<float, KL_KERNEL_ADVEC_U_2I5>
                                                            : &launch_plain<float, KL_KERNEL_DIFF_SMAG>,
                            nullptr, nullptr});
        add_variants_f32_les(kernel, v);
        return v;
    }
    v.push_back(Variant{"default", kernel, KL_F32, FAMILY_PLAIN, 1, 256, 1, 1, 0,
                        kernel == KL_KERNEL_ADVEC_U ? &launch_plain<float, KL_KERNEL_ADVEC_U>
                                                    : &launch_plain<float, KL_KERNEL_DIFF_UVW>,
                        nullptr, nullptr});
        add_variants_f32_zc(kernel, v);
        add_variants_f32_zl1(kernel, v);
        add_variants_f32_zl2(kernel, v);
        add_variants_f32_zl4(kernel, v);
        add_variants_f32_x(kernel, v);
        add_variants_f32_nt(kernel, v);
        add_variants_f32_small(kernel, v);
        add_variants_f32_rev(kernel, v);
        if (kernel == KL_KERNEL_DIFF_UVW) add_variants_f32_split(v);
    return v;
}

const std::vector<Variant> &variants_f32(int kernel)
{
    static const std::vector<Variant> advec = build_f32(KL_KERNEL_ADVEC_U);
    static const std::vector<Variant> diff = build_f32(KL_KERNEL_DIFF_UVW);
    static const std::vector<Variant> step = build_f32(KL_KERNEL_STEP);
    static const std::vector<Variant> advec5 = build_f32(KL_KERNEL_ADVEC_U_2I5);
    static const std::vector<Variant> smag = build_f32(KL_KERNEL_DIFF_SMAG);
    static const std::vector<Variant> ad = build_f32(KL_KERNEL_ADVEC_DIFF);
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
