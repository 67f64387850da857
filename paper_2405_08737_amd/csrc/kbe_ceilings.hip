// Ceiling microbenchmarks: the FP64 matrix-core and HBM rates this GPU actually sustains, against
// which the library's kernels are measured (the published peaks are 78.6 TFLOP/s and 8 TB/s).
//
//   mfma 4x4x4   : every wave issues chains of independent v_mfma_f64_4x4x4 products (four 4x4x4
//                  blocks per instruction, 512 FLOP), 8 accumulators in flight;
//   mfma 16x16x4 : the same with v_mfma_f64_16x16x4 (2048 FLOP per instruction);
//   read         : a grid-stride stream of 16-byte loads over a buffer, summed per thread;
//   copy         : the same stream stored to a second buffer.
// The caller times the launches (HIP events on the stream) and divides the counts returned by
// kbe_internal_ceiling_counts by the time.  Results are stored so no work is dead.
#include "kbe_dev.h"
#include "kbe_internal.h"

namespace kbe {
namespace {

typedef double __attribute__((ext_vector_type(4))) d4c;

constexpr int CHAINS = 8;
constexpr int GRID = 2048, BLOCK = 256;  // 8 waves per CU over 256 CUs

__global__ void __launch_bounds__(BLOCK) ceil_mfma4(double *out, int iters, double seed) {
  double acc[CHAINS];
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) acc[c] = c * 1e-3;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += acc[c];
  out[(int64_t)blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) ceil_mfma16(double *out, int iters, double seed) {
  d4c acc[CHAINS];
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) acc[c] = d4c{c * 1e-3, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += acc[c].x + acc[c].y + acc[c].z + acc[c].w;
  out[(int64_t)blockIdx.x * BLOCK + threadIdx.x] = s;
}

__global__ void __launch_bounds__(BLOCK) ceil_read(const double2 *src, int64_t n2, double *out) {
  double2 s = make_double2(0.0, 0.0);
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n2; i += stride) {
    const double2 v = src[i];
    s.x += v.x;
    s.y += v.y;
  }
  out[(int64_t)blockIdx.x * BLOCK + threadIdx.x] = s.x + s.y;
}

__global__ void __launch_bounds__(BLOCK) ceil_copy(const double2 *src, double2 *dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace kbe

// Declared in kbe_internal.h.
extern "C" int32_t kbe_internal_ceiling_run(int32_t kind, const void *src, void *dst,
                                            int64_t bytes, double *out, int32_t iters,
                                            void *stream) {
  using namespace kbe;
  hipStream_t st = (hipStream_t)stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(ceil_mfma4, dim3(GRID), dim3(BLOCK), 0, st, out, iters, 1.0); break;
    case 1: hipLaunchKernelGGL(ceil_mfma16, dim3(GRID), dim3(BLOCK), 0, st, out, iters, 1.0); break;
    case 2:
      hipLaunchKernelGGL(ceil_read, dim3(GRID), dim3(BLOCK), 0, st, (const double2 *)src,
                         bytes / 16, out);
      break;
    case 3:
      hipLaunchKernelGGL(ceil_copy, dim3(GRID), dim3(BLOCK), 0, st, (const double2 *)src,
                         (double2 *)dst, bytes / 16);
      break;
    default: return 1;
  }
  return hipGetLastError() == hipSuccess ? 0 : 4;
}

// FLOP (kinds 0, 1) or HBM bytes (kinds 2: read; 3: read + written) of one launch.
extern "C" double kbe_internal_ceiling_counts(int32_t kind, int64_t bytes, int32_t iters) {
  using namespace kbe;
  const double instr = (double)GRID * (BLOCK / 64) * iters * CHAINS;  // per wave: iters x chains
  switch (kind) {
    case 0: return instr * 512.0;
    case 1: return instr * 2048.0;
    case 2: return (double)bytes;
    case 3: return 2.0 * (double)bytes;
    default: return 0.0;
  }
}

// Size of the `out` array the launches write (doubles).
extern "C" int64_t kbe_internal_ceiling_out_count(void) { return (int64_t)kbe::GRID * kbe::BLOCK; }
