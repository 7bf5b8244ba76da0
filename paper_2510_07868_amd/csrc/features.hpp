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
  f[9] = 2.0f * (sqrtf(t.x) - 1.0f);
  f[10] = 2.0f * (sqrtf(t.y) - 1.0f);
  f[11] = 2.0f * (sqrtf(t.z) - 1.0f);
  f[12] = m0.x;
  f[13] = m0.y;
  f[14] = m0.z;
  f[15] = 1.0f - expf(-(type == 1u ? m0.w : 1.0f));
  f[16] = (float)depth / (float)max_depth;
  const float w = 16.0f * 3.14159265358979f;
  f[17] = sinf(w * pn.x);
  f[18] = sinf(w * pn.y);
  f[19] = sinf(w * pn.z);
}

}  // namespace nrrs
