// Shared pieces of the pair-block kernels (pntile.hip: proton-neutron part; flytile.hip:
// single-species two-body part): the matrix-core instruction per precision and its output layout,
// the sign flip, the work-item order and the gathers of one group of source rows.
#pragma once
#include "internal.h"

namespace trbl {
namespace tiles {

// Per precision: the matrix-core accumulator, the instruction, and the row of its output a lane
// register holds (measured on gfx950: FP64 D[l / 16 + 4 v][l % 16], FP32 D[4 (l / 16) + v][l % 16]).
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
  static constexpr unsigned ZSHIFT = 7;  // bytes of a 16-value row: 128
};
template <>
struct Mfma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
  static constexpr unsigned ZSHIFT = 6;  // 64
};

constexpr int PN_TPB = 256;       // most core pairs of one work item
constexpr int PN_MAXPAIR = 64;    // widest pair block (one ballot)

// work item -> position: consecutive items (one proton core) go to one XCD
__device__ __forceinline__ int pn_xcd_item(int bid, int n) {
  const int per = (n + 7) / 8;
  return (bid % 8) * per + bid / 8;
}

__device__ __forceinline__ double flip_if(double x, unsigned s) {
  return __hiloint2double(__double2hiint(x) ^ (int)(s << 31), __double2loint(x));
}
__device__ __forceinline__ float flip_if(float x, unsigned s) { return __int_as_float(__float_as_int(x) ^ (int)(s << 31)); }

template <class T>
__device__ __forceinline__ void tile_loads(const unsigned* Rv, int h, int kq, unsigned cb, const char* Vb,
                                           T (&bop)[8]) {
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const unsigned o = Rv[4 * (8 * h + j) + kq];
    bop[j] = *reinterpret_cast<const T*>(Vb + ((o & ~1u) + cb));
  }
}

inline int64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long double r = 1.0L;
  for (int i = 0; i < k; i++) r = r * (n - i) / (i + 1);
  return (int64_t)(r + 0.5L);
}


}  // namespace tiles
}  // namespace trbl
