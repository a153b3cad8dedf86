// store.h -- population storage formats.
//
// Layout: structure of arrays, one plane per (set, i) holding that population
// for every node in x-fastest order, so a wavefront of consecutive x reads one
// contiguous run per population (pull streaming shifts it by at most one).
//
// Values kept (Sec. 3.1, eq. EDF): for f the deviation f_i - w_i rho0 from
// the weight times a reference density (f_i is w_i p/c_s^2 (1 + O(u)) for
// i > 0, p the lattice pressure, which is c_s^2 rho0 up to O(1e-3) in every
// phase -- rho0 = 1 for equal component densities, (M_1 + M_2)/2 otherwise --
// so the deviation keeps the velocity-carrying part at full relative
// precision; f_0 carries the density contrast between phases); for g and h the
// populations themselves.  The moving populations g_i, h_i (i > 0) are
// O(mu, u) and small, while the rest populations g_0 and h_0 carry the order
// parameters phi in [-1, 1] and psi in [0, 1].  Their rounding is what limits
// a single-precision run: the Laplacian and then the gradient of the
// chemical potential amplify it by an order of magnitude before it reaches
// the force.  The mixed format therefore keeps g_0 and h_0 in FP64 and
// everything else in FP32.
//
// Interface of every format:
//   load<R>(set, i, node)      moving population (or f_0), as R
//   rest(set, node)            g_0 / h_0 (set 1, 2) as double, f_0 for set 0
//   store<R>(set, i, node, v)  moving population (or f_0)
//   store_rest(set, node, v)   g_0 / h_0
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.h"

namespace lb {

typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

// all planes in one type T (FP32 or FP64): p[(set * Q + i) * N + node]
template <typename T, int Q>
struct PlainStore {
  T* p;
  long long N;
  template <typename R>
  __device__ __forceinline__ R load(int set, int i, long long node) const {
    return (R)p[((long long)(set * Q + i)) * N + node];
  }
  __device__ __forceinline__ double rest(int set, long long node) const {
    return (double)p[((long long)(set * Q)) * N + node];
  }
  template <typename R>
  __device__ __forceinline__ void store(int set, int i, long long node, R v) const {
    p[((long long)(set * Q + i)) * N + node] = (T)v;
  }
  __device__ __forceinline__ void store_rest(int set, long long node, double v) const {
    p[((long long)(set * Q)) * N + node] = (T)v;
  }
  static constexpr bool kQuantized = false;
  template <typename R>
  __device__ __forceinline__ R quantize(R v) const { return v; }
  static constexpr long long bytes_per_node() { return 3LL * Q * (long long)sizeof(T); }
};

// FP32 planes for f_0..f_{Q-1}, g_1.., h_1..; FP64 planes for g_0 and h_0.
//   f_i:   p[i * N + node]
//   g_i:   p[(Q + i - 1) * N + node]          i >= 1
//   h_i:   p[(2Q - 1 + i - 1) * N + node]     i >= 1
//   g_0:   r[node], h_0: r[N + node]
// (The buffer builtins move raw 32/64-bit words; values are bit-cast.)
// Accesses go through buffer resources: the plane offset is a uniform
// (scalar) byte offset and the node a 32-bit per-lane offset, so one address
// register serves the three populations that travel along the same link.
// The FP32 planes of one buffer must stay below 4 GiB (checked on the host).
template <int Q>
struct MixStore {
  float* p;
  double* r;
  long long N;
  __device__ __forceinline__ static long long plane(int set, int i) {
    return set == 0 ? i : (set == 1 ? Q + i - 1 : 2 * Q - 1 + i - 1);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rp() const {
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)0xffffffffu, 0x00020000);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rr() const {
    return __builtin_amdgcn_make_buffer_rsrc(r, 0, (int)0xffffffffu, 0x00020000);
  }
  template <typename R>
  __device__ __forceinline__ R load(int set, int i, long long node) const {
    if (set > 0 && i == 0) return (R)rest(set, node);
    return (R)__builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(rp(), (int)(node * 4), (int)(plane(set, i) * N * 4), 0));
  }
  __device__ __forceinline__ double rest(int set, long long node) const {
    if (set == 0)
      return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp(), (int)(node * 4), 0, 0));
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                          rr(), (int)(node * 8), (int)((long long)(set - 1) * N * 8), 0));
  }
  template <typename R>
  __device__ __forceinline__ void store(int set, int i, long long node, R v) const {
    if (set > 0 && i == 0) {
      store_rest(set, node, (double)v);
      return;
    }
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)v), rp(), (int)(node * 4),
                                          (int)(plane(set, i) * N * 4), 0);
  }
  __device__ __forceinline__ void store_rest(int set, long long node, double v) const {
    if (set == 0) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)v), rp(), (int)(node * 4), 0,
                                            0);
      return;
    }
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rr(), (int)(node * 8),
                                          (int)((long long)(set - 1) * N * 8), 0);
  }
  static constexpr bool kQuantized = false;
  template <typename R>
  __device__ __forceinline__ R quantize(R v) const { return v; }
  static constexpr long long float_planes() { return 3LL * Q - 2; }
  static constexpr long long bytes_per_node() { return float_planes() * 4 + 2 * 8; }
};

// 16-bit moving populations; the rest population f_0 - w_0 in FP32 and g_0,
// h_0 in FP64, as in the mixed format.  Moving values are multiplied by a
// fixed power of two before rounding so that typical magnitudes (1e-6 ..
// 1e-2) stay clear of the half subnormal range; bf16 uses the same scale
// (its exponent range makes it harmless).  The collision adds each moving
// population's rounding to the rest population of its node and set, so
// every set's mass survives the rounding.  g_0 and h_0 are O(1) (they carry
// phi and psi), and an FP32 rest population near 1 would drop additions
// below half its ulp every step, a steady drift of the order parameters'
// totals; in FP64 those additions are kept.
//   mov[(set * (Q-1) + i - 1) * N + node]   i = 1..Q-1
//   r0[node]                                 f_0 - w_0
//   r12[(set - 1) * N + node]                g_0 (set 1), h_0 (set 2)
template <typename H, int Q>
struct Split16Store {
  H* mov;
  float* r0;
  double* r12;
  long long N;
  static constexpr float kScale = 1024.0f;
  static constexpr float kInv = 1.0f / 1024.0f;
  template <typename R>
  __device__ __forceinline__ R load(int set, int i, long long node) const {
    if (i == 0) return (R)rest(set, node);
    return (R)(to_float(mov[((long long)(set * (Q - 1) + i - 1)) * N + node]) * kInv);
  }
  __device__ __forceinline__ double rest(int set, long long node) const {
    return set == 0 ? (double)r0[node] : r12[(long long)(set - 1) * N + node];
  }
  template <typename R>
  __device__ __forceinline__ void store(int set, int i, long long node, R v) const {
    if (i == 0)
      store_rest(set, node, (double)v);
    else
      mov[((long long)(set * (Q - 1) + i - 1)) * N + node] = from_float((float)v * kScale);
  }
  __device__ __forceinline__ void store_rest(int set, long long node, double v) const {
    if (set == 0)
      r0[node] = (float)v;
    else
      r12[(long long)(set - 1) * N + node] = v;
  }
  // the value a moving population reads back as after a store
  static constexpr bool kQuantized = true;
  template <typename R>
  __device__ __forceinline__ R quantize(R v) const {
    return (R)(to_float(from_float((float)v * kScale)) * kInv);
  }
  __device__ static __forceinline__ float to_float(__half h) { return __half2float(h); }
  __device__ static __forceinline__ float to_float(__hip_bfloat16 h) { return __bfloat162float(h); }
  __device__ static __forceinline__ H from_float(float f);
  static constexpr long long bytes_per_node() {
    return 3LL * (Q - 1) * (long long)sizeof(H) + 4 + 2 * 8;
  }
};

template <>
__device__ __forceinline__ __half Split16Store<__half, 9>::from_float(float f) {
  return __float2half_rn(f);
}
template <>
__device__ __forceinline__ __half Split16Store<__half, 19>::from_float(float f) {
  return __float2half_rn(f);
}
template <>
__device__ __forceinline__ __hip_bfloat16 Split16Store<__hip_bfloat16, 9>::from_float(float f) {
  return __float2bfloat16(f);
}
template <>
__device__ __forceinline__ __hip_bfloat16 Split16Store<__hip_bfloat16, 19>::from_float(float f) {
  return __float2bfloat16(f);
}

}  // namespace lb
