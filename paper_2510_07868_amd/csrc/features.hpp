// The 20 network inputs at a path vertex: position in the scene box, face-forwarded normal,
// outgoing direction, Box-Cox(lambda = 0.5) throughput and remapped roughness as in the
// paper's input encodings (Sec. 5 "Input Encoding"), albedo, relative depth and one octave
// of sine-encoded position.
#pragma once
#include "device_common.hpp"

namespace nrrs {

__device__ __forceinline__ void vertex_features(const DevScene& sc, V3 p, V3 n, V3 wo, V3 t, float4 m0,
                                                uint32_t type, uint32_t depth, uint32_t max_depth, float f[20]) {
  const float inv_ext = 1.0f / sc.extent;
  const V3 pn = v3((p.x - sc.amin_x) * inv_ext, (p.y - sc.amin_y) * inv_ext, (p.z - sc.amin_z) * inv_ext);
  f[0] = 2.0f * pn.x - 1.0f;
  f[1] = 2.0f * pn.y - 1.0f;
  f[2] = 2.0f * pn.z - 1.0f;
  f[3] = n.x;
  f[4] = n.y;
  f[5] = n.z;
  f[6] = wo.x;
  f[7] = wo.y;
  f[8] = wo.z;
  // hardware square root, exponential and sine: a network input needs no correctly rounded
  // value, and the library versions cost the inference kernel a fifth of its vector
  // instructions (the sine's argument reduction above all)
  f[9] = 2.0f * (__builtin_amdgcn_sqrtf(t.x) - 1.0f);
  f[10] = 2.0f * (__builtin_amdgcn_sqrtf(t.y) - 1.0f);
  f[11] = 2.0f * (__builtin_amdgcn_sqrtf(t.z) - 1.0f);
  f[12] = m0.x;
  f[13] = m0.y;
  f[14] = m0.z;
  f[15] = 1.0f - __builtin_amdgcn_exp2f(-1.44269504088896341f * (type == 1u ? m0.w : 1.0f));
  f[16] = (float)depth / (float)max_depth;
  // sin(16 pi x) = sin(2 pi (8 x)): the hardware sine takes its argument in turns
  f[17] = __builtin_amdgcn_sinf(8.0f * pn.x);
  f[18] = __builtin_amdgcn_sinf(8.0f * pn.y);
  f[19] = __builtin_amdgcn_sinf(8.0f * pn.z);
}

// Network factor at a vertex: the ADRRS ratio of the throughput's luminance lt times the
// predicted reflected radiance y to the pixel estimate g (Sec. 2.2; + 0.01 as in the relative
// error), held within [q_h / 8, 64 q_h] of the heuristic factor q_h of the same vertex.  An
// estimate far below the truth (the network's output shrinks toward 0 where most training
// targets are 0, e.g. a room lit through a small opening) would otherwise give the rare
// surviving path a weight of 1 / q that is orders of magnitude too large; any positive factor
// keeps the estimator unbiased.  A non-finite ratio keeps the heuristic factor.
__device__ __forceinline__ float network_factor(float lt, float y, float g, float q_h) {
  const float q = lt * y / (g + 0.01f);
  if (!isfinite(q)) return q_h;
  return fminf(fmaxf(q, 0.125f * q_h), 64.0f * q_h);
}

}  // namespace nrrs
