// Device-side definitions shared by the HIP kernels of libkbe (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kbe.h"

namespace kbe {

struct cd {  // complex double in registers
  double re, im;
};

__device__ __forceinline__ cd ld(const kbe_c128 *p) {
  // 16-byte load of one complex128
  const double2 v = *reinterpret_cast<const double2 *>(p);
  return {v.x, v.y};
}
__device__ __forceinline__ void st(kbe_c128 *p, cd v) {
  *reinterpret_cast<double2 *>(p) = make_double2(v.re, v.im);
}
// The same through a pointer known to address global memory (for pointers rebuilt from integers,
// e.g. after readfirstlane, whose address space the compiler can no longer infer; a generic
// pointer would turn the access into a flat one that also counts against the LDS wait counter).
typedef double __attribute__((ext_vector_type(2))) dvec2;
typedef __attribute__((address_space(1))) dvec2 g_dvec2;
__device__ __forceinline__ cd ldg(const kbe_c128 *p) {
  const dvec2 v = *(const g_dvec2 *)(const void *)p;
  return {v.x, v.y};
}
__device__ __forceinline__ void stg(kbe_c128 *p, cd v) {
  dvec2 w;
  w.x = v.re;
  w.y = v.im;
  *(g_dvec2 *)(void *)p = w;
}
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator-(cd a) { return {-a.re, -a.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cd cj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ cd czero() { return {0.0, 0.0}; }

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also orders global memory,
// which makes every wave wait for all of its outstanding global loads (prefetches included).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Every pointer/size a collision-type kernel can need.  Passed by value.
struct Params {
  int N, nt, ntau, J, n, m0, m1;
  int64_t ldt;
  const kbe_c128 *kp, *rdiag, *tv, *mat;       // Green's function
  const kbe_c128 *ret, *les, *stv;             // self-energy row at t_n
  const kbe_c128 *sgt;                         // Sigma^> row (both forms in one call)
  const double *w, *wtau, *wf;                 // weights
  const kbe_c128 *gIR, *gIL, *gItv, *gJ;       // cotangents (adjoint only)
  kbe_c128 *gkp, *grdiag, *gtv;                // gradient outputs (adjoint only)
  int overwrite;                               // adjoint: overwrite instead of accumulate
  int fIR, fIL, fITV, fJTV;                    // selected outputs
};

__host__ __device__ __forceinline__ int64_t bsz(const Params &p) { return (int64_t)p.N * p.N; }
__host__ __device__ __forceinline__ const kbe_c128 *kp_blk(const Params &p, int a, int b) {
  return p.kp + ((int64_t)a * p.ldt + b) * bsz(p);
}
__host__ __device__ __forceinline__ const kbe_c128 *tv_blk(const Params &p, int m, int j) {
  return p.tv + ((int64_t)m * p.ntau + j) * bsz(p);
}

}  // namespace kbe
