// Mix-Depth's fixed-rate method (Sec. 4.3): at a depth assigned to it, every vertex that
// continues gets the same raw factor, so the per-depth normalization (Sec. 4.1 Eqs. 9-10)
// gives all paths one survival / splitting rate.  Runs after shading, in place of the network.
#include <algorithm>

#include "launch.hpp"

namespace nrrs {

namespace {

constexpr int kFixedThreads = 256;

__global__ __launch_bounds__(kFixedThreads) void k_fixed_factor(RenderArgs a) {
  const uint32_t n = a.ctl[a.depth].n;
  for (uint32_t i = blockIdx.x * kFixedThreads + threadIdx.x; i < n; i += gridDim.x * kFixedThreads)
    a.q[i] = a.q[i] > 0.0f ? 1.0f : 0.0f;
}

}  // namespace

void launch_fixed_factor(const RenderArgs& a, hipStream_t s) {
  const uint32_t blocks = std::min<uint32_t>((a.cap + kFixedThreads - 1) / kFixedThreads, 8192u);
  hipLaunchKernelGGL(k_fixed_factor, dim3(std::max<uint32_t>(blocks, 1u)), dim3(kFixedThreads), 0, s, a);
}

}  // namespace nrrs
