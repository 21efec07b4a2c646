// multi.hpp -- one launch for many simulations.  A launch takes a table of
// ops (one simulation's kernel arguments together with the kernel body they
// run) and each op's first block; block b runs the op whose block range holds
// b, with its block index inside that range, so every block belongs to one
// simulation and sees exactly what its own single-simulation launch would.
// Included by amr.hpp.
#pragma once
#include <hip/hip_runtime.h>

namespace mdlts {

// The op of block blockIdx.x: the last entry of the ascending first-block
// table not above it (the same on every lane of the wave), found with one
// load per 64 entries and a ballot.
__device__ __forceinline__ int multi_entry(const int *__restrict__ block0, int n)
{
    const int lane = (int)(threadIdx.x & 63);
    const int b = (int)blockIdx.x;
    int q = 0;
    for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        const unsigned long long m = __ballot(i < n && block0[i] <= b);
        const int c = __popcll(m);
        if (c == 0) break;
        q = base + c - 1;
        if (c < 64) break;
    }
    return __builtin_amdgcn_readfirstlane(q);
}

template <typename Op>
__global__ __launch_bounds__(256) void k_multi(const Op *__restrict__ ops, const int *__restrict__ block0, int n)
{
    const int q = multi_entry(block0, n);
    const Op &op = ops[q];
    op((int)blockIdx.x - block0[q]);
}

}  // namespace mdlts
