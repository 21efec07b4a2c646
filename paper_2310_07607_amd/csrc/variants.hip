// variants.hip -- the substep kernels of one polynomial degree
// (MDLTS_DEGREE), both launch forms, both precisions, diagonal and full
// diffusion tensors.
#include "kernels.hpp"
#include "variants.hpp"

#ifndef MDLTS_DEGREE
#error "compile with -DMDLTS_DEGREE=1, 2 or 3"
#endif

namespace mdlts {

namespace {

template <int DIM, typename T, bool FULL>
void *pick(int form)
{
    if (form == kFormBatch) return reinterpret_cast<void *>(&k_substep_batch<DIM, MDLTS_DEGREE, T, FULL>);
    return reinterpret_cast<void *>(&k_substep<DIM, MDLTS_DEGREE, T, FULL>);
}

template <int DIM>
void *pick_dim(int form, bool fp32, bool full)
{
    if (fp32) return full ? pick<DIM, float, true>(form) : pick<DIM, float, false>(form);
    return full ? pick<DIM, double, true>(form) : pick<DIM, double, false>(form);
}

}  // namespace

template <>
void *substep_kernel<MDLTS_DEGREE>(int form, int dim, bool fp32, bool full)
{
    if (dim == 2) return pick_dim<2>(form, fp32, full);
    if (dim == 3) return pick_dim<3>(form, fp32, full);
    return nullptr;
}

}  // namespace mdlts
