// Grid-row helpers shared by the forward and adjoint row-sharing stencil
// kernels (device code).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mono {

template <typename T>
__device__ __forceinline__ T ld_bytes(const T* base, uint32_t byte_off) {
  return *(const T*)((const char*)base + byte_off);
}

// On a structured grid numbered x fastest the stencil offsets come in
// triples c-1, c, c+1 around a few "row centres" c (0 and +-nx in 2D; 0,
// +-nx, +-(nxy-nx), +-nxy, +-(nxy+nx) in 3D).  A wavefront then loads each
// centre row once for its 64 consecutive rows and takes the x-1 / x+1
// neighbours from the adjacent lanes (DPP wavefront shifts); lanes 0 and 63
// only supply those neighbours, lanes 1..62 produce rows.  RowPattern<P> maps
// the forward (i + off_p) and backward (i - off_p) neighbour of slot p to a
// centre k and a lane shift d.
template <int P>
struct RowPattern;
template <>
struct RowPattern<1> {
  static constexpr int NC = 1;
  __device__ static constexpr int fk(int) { return 0; }
  __device__ static constexpr int fd(int) { return 1; }
  __device__ static constexpr int bk(int) { return 0; }
  __device__ static constexpr int bd(int) { return -1; }
};
template <>
struct RowPattern<4> {   // centres 0, +nx, -nx; offsets 1, nx-1, nx, nx+1
  static constexpr int NC = 3;
  __device__ static constexpr int fk(int p) { return p == 0 ? 0 : 1; }
  __device__ static constexpr int fd(int p) { return p == 0 ? 1 : p - 2; }
  __device__ static constexpr int bk(int p) { return p == 0 ? 0 : 2; }
  __device__ static constexpr int bd(int p) { return p == 0 ? -1 : 2 - p; }
};
template <>
struct RowPattern<13> {  // centres 0, nx, nxy-nx, nxy, nxy+nx, then their negatives
  static constexpr int NC = 9;
  __device__ static constexpr int fk(int p) { return p == 0 ? 0 : 1 + (p - 1) / 3; }
  __device__ static constexpr int fd(int p) { return p == 0 ? 1 : (p - 1) % 3 - 1; }
  __device__ static constexpr int bk(int p) { return p == 0 ? 0 : 5 + (p - 1) / 3; }
  __device__ static constexpr int bd(int p) { return p == 0 ? -1 : 1 - (p - 1) % 3; }
};

// value of the next (d = 1) or previous (d = -1) lane of the wavefront; the
// lane with no such neighbour reads 0 (bound_ctrl set: no zero-initialised
// destination needed)
template <int D, typename T>
__device__ __forceinline__ T lane_shift(T v) {
  if constexpr (D == 0) {
    return v;
  } else if constexpr (sizeof(T) == 4) {
    const int x = __builtin_amdgcn_update_dpp(0, __float_as_int(v), D > 0 ? 0x130 : 0x138, 0xf,
                                              0xf, true);
    return __int_as_float(x);
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), D > 0 ? 0x130 : 0x138,
                                               0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), D > 0 ? 0x130 : 0x138, 0xf,
                                               0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
}

}  // namespace mono
