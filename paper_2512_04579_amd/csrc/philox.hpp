// Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller transforms that
// turn one Philox block into normal draws, shared by the sampler (sample.hip)
// and the rollout that draws its own perturbations (rollout.hip), so that both
// produce bit-identical W.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gnm {
namespace {

struct Philox4x32 {
  uint32_t c0, c1, c2, c3;
};

__device__ __forceinline__ Philox4x32 philox4x32_10(Philox4x32 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
  constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(kMul0, c.c0), lo0 = kMul0 * c.c0;
    const uint32_t hi1 = __umulhi(kMul1, c.c2), lo1 = kMul1 * c.c2;
    c = Philox4x32{hi1 ^ c.c1 ^ k0, lo1, hi0 ^ c.c3 ^ k1, lo0};
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// Box-Muller from two 32-bit words: u1 in (0, 1] (never 0, so the log is
// finite), u2 in [0, 1).  24-bit uniforms are exact in float.
__device__ __forceinline__ void box_muller_f32(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float u1 = static_cast<float>((a >> 8) + 1u) * 0x1.0p-24f;
  const float u2 = static_cast<float>(b >> 8) * 0x1.0p-24f;
  const float rad = __builtin_sqrtf(-2.0f * logf(u1));
  float s, c;
  sincospif(2.0f * u2, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

__device__ __forceinline__ void box_muller_f64(Philox4x32 x, double& z0, double& z1) {
  const uint64_t a = (static_cast<uint64_t>(x.c0) << 21) | (x.c1 >> 11);
  const uint64_t b = (static_cast<uint64_t>(x.c2) << 21) | (x.c3 >> 11);
  const double u1 = static_cast<double>(a + 1u) * 0x1.0p-53;
  const double u2 = static_cast<double>(b) * 0x1.0p-53;
  const double rad = __builtin_sqrt(-2.0 * log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// The normals of Philox block b at draw column s times sigma: FP32 rows
// 4 b .. 4 b + 3 (words (c0, c1) and (c2, c3)), FP64 rows 2 b, 2 b + 1.  The
// products are not contracted with anything that follows.
template <typename T>
constexpr int philox_rows() {
  return sizeof(T) == 4 ? 4 : 2;
}

template <typename T>
__device__ __forceinline__ void scaled_normals(uint32_t s, uint32_t b, uint32_t k0, uint32_t k1,
                                               uint32_t s0, uint32_t s1, T sigma,
                                               T (&v)[philox_rows<T>()]) {
#pragma clang fp contract(off)
  const Philox4x32 x = philox4x32_10(Philox4x32{s, b, s0, s1}, k0, k1);
  T z[philox_rows<T>()];
  if constexpr (sizeof(T) == 4) {
    box_muller_f32(x.c0, x.c1, z[0], z[1]);
    box_muller_f32(x.c2, x.c3, z[2], z[3]);
  } else {
    box_muller_f64(x, z[0], z[1]);
  }
#pragma unroll
  for (int t = 0; t < philox_rows<T>(); ++t) v[t] = sigma * z[t];
}

}  // namespace
}  // namespace gnm
