// variants.hpp -- host addresses of the substep kernels, one translation
// unit per polynomial degree (variants.hip compiled with MDLTS_DEGREE = 1, 2,
// 3), so that the kernel variants compile in parallel.
#pragma once

namespace mdlts {

enum SubstepForm { kFormBatch = 0, kFormEager = 1 };

// The kernel k_substep_batch<dim, P, T, full> (kFormBatch) or
// k_substep<dim, P, T, full> (kFormEager), T = float if fp32 else double;
// nullptr for a dimension other than 2 or 3.
template <int P>
void *substep_kernel(int form, int dim, bool fp32, bool full);
template <>
void *substep_kernel<1>(int form, int dim, bool fp32, bool full);
template <>
void *substep_kernel<2>(int form, int dim, bool fp32, bool full);
template <>
void *substep_kernel<3>(int form, int dim, bool fp32, bool full);

inline void *substep_kernel_of(int form, int dim, int order, bool fp32, bool full)
{
    switch (order) {
    case 1: return substep_kernel<1>(form, dim, fp32, full);
    case 2: return substep_kernel<2>(form, dim, fp32, full);
    case 3: return substep_kernel<3>(form, dim, fp32, full);
    }
    return nullptr;
}

}  // namespace mdlts
