// Device helpers shared by the solver kernels: wavefront reductions with DPP,
// workgroup reductions, and loads that pick the address space (per-scenario
// arrays through the global space with 32-bit offsets, network data through
// the constant space).
#pragma once

#include <hip/hip_runtime.h>

namespace pfx {

constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sum over the 64 lanes of a wave with DPP row operations (no LDS traffic):
// quad swaps, half-row and row mirrors, then the row broadcasts; the total
// ends in lane 63 and is returned to every lane through a scalar register.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float wave_total(float v) {
  v += dpp_f<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_f<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_f<0x140, 0xf>(v);  // row_mirror
  v += dpp_f<0x142, 0xa>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_f<0x143, 0xc>(v);  // row_bcast31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_total(double v) {
  v += dpp_d<0xB1, 0xf>(v);
  v += dpp_d<0x4E, 0xf>(v);
  v += dpp_d<0x141, 0xf>(v);
  v += dpp_d<0x140, 0xf>(v);
  v += dpp_d<0x142, 0xa>(v);
  v += dpp_d<0x143, 0xc>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// max that propagates NaN
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)); }
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// The network descriptor is re-read at the start of each phase: hiding the
// pointer's value from the optimiser keeps the descriptor's ~50 fields from
// being held in registers across the whole kernel, and reading it through the
// constant address space keeps the reads scalar (only the fields a phase uses
// are loaded).
template <typename P>
__device__ __forceinline__ P load_desc(const P* p) {
  static_assert(sizeof(P) % 8 == 0, "descriptor size");
  asm volatile("" : "+s"(p));
  typedef __attribute__((address_space(4))) const unsigned long long CU;
  unsigned long long words[sizeof(P) / 8];
#pragma unroll
  for (unsigned i = 0; i < sizeof(P) / 8; ++i) words[i] = ((CU*)p)[i];
  P out;
  __builtin_memcpy(&out, words, sizeof(P));
  return out;
}

// Workgroup sum into every thread.  `part` (NW entries) must not be written
// again before the next barrier: callers alternate between two buffers.
template <typename T, int BLOCK>
__device__ T block_sum(T v, T* part) {
  constexpr int NW = BLOCK / WAVE;
  v = wave_total(v);
  if (lane_id() == 0) part[wave_id()] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += part[i];
  return s;
}

template <int BLOCK>
__device__ double block_nanmax(double v, double* part) {
  constexpr int NW = BLOCK / WAVE;
  v = wave_nanmax(v);
  if (lane_id() == 0) part[wave_id()] = v;
  __syncthreads();
  double s = part[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = nanmax(s, part[i]);
  return s;
}

// Per-scenario data: element access by a 32-bit index from a base pointer that
// is uniform across the workgroup (global address space, scalar base plus a
// 32-bit vector offset).
template <typename T>
__device__ __forceinline__ T gld(const T* base, unsigned i) {
  typedef __attribute__((address_space(1))) const char GC;
  typedef __attribute__((address_space(1))) const T GT;
  return *(GT*)((GC*)base + i * (unsigned)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void gst(T* base, unsigned i, T v) {
  typedef __attribute__((address_space(1))) char GC;
  typedef __attribute__((address_space(1))) T GT;
  *(GT*)((GC*)base + i * (unsigned)sizeof(T)) = v;
}

// Network data: read-only for the whole launch, so it is read through the
// constant address space (scalar loads at uniform indexes, free scheduling).
template <typename T>
__device__ __forceinline__ T cld(const T* base, unsigned i) {
  typedef __attribute__((address_space(4))) const char CC;
  typedef __attribute__((address_space(4))) const T CT;
  return *(CT*)((CC*)base + i * (unsigned)sizeof(T));
}

// complex entries: one 16- (or 8-) byte load of the native two-element vector
__device__ __forceinline__ double2 cld(const double2* base, unsigned i) {
  typedef double __attribute__((ext_vector_type(2))) D2;
  typedef __attribute__((address_space(4))) const char CC;
  typedef __attribute__((address_space(4))) const D2 CT;
  const D2 v = *(CT*)((CC*)base + i * 16u);
  double2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

__device__ __forceinline__ float2 cld(const float2* base, unsigned i) {
  typedef float __attribute__((ext_vector_type(2))) F2;
  typedef __attribute__((address_space(4))) const char CC;
  typedef __attribute__((address_space(4))) const F2 CT;
  const F2 v = *(CT*)((CC*)base + i * 8u);
  float2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

// For a kernel whose workgroup is a single wavefront and whose lanes exchange
// data through LDS only: waits for the wavefront's own LDS operations, so
// its later LDS reads see every lane's earlier writes, without the wait for
// outstanding global loads that __syncthreads() implies (a workgroup-scope
// fence), which would stall on loads issued ahead for the next step.  The
// memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Compiler-only fence between the bus slots of an unrolled loop: keeps the
// loads of later slots from being hoisted above earlier ones, which would hold
// every slot's operands in registers at once.
__device__ __forceinline__ void slot_fence() { asm volatile("" ::: "memory"); }

// Forces a value to be computed at this point (it cannot be sunk below), so a
// slot's result does not keep its operands alive through the later slots.
template <typename T>
__device__ __forceinline__ void settle(T& x) {
  asm volatile("" : "+v"(x));
}

__device__ __forceinline__ int2 cld(const int2* base, unsigned i) {
  typedef int __attribute__((ext_vector_type(2))) I2;
  typedef __attribute__((address_space(4))) const char CC;
  typedef __attribute__((address_space(4))) const I2 CT;
  const I2 v = *(CT*)((CC*)base + i * 8u);
  int2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

__device__ __forceinline__ int4 cld(const int4* base, unsigned i) {
  typedef int __attribute__((ext_vector_type(4))) I4;
  typedef __attribute__((address_space(4))) const char CC;
  typedef __attribute__((address_space(4))) const I4 CT;
  const I4 v = *(CT*)((CC*)base + i * 16u);
  int4 r;
  r.x = v.x;
  r.y = v.y;
  r.z = v.z;
  r.w = v.w;
  return r;
}

}  // namespace pfx
