// Matrix-core rate probes: the instruction of the INT8 slice products
// (v_mfma_i32_16x16x64_i8) and that of the FP64 plain form
// (v_mfma_f64_16x16x4_f64) issued back to back from registers by every
// wavefront of a grid that fills the chip, with no memory traffic, so that
// the slice GEMM's achieved rate can be set against what the hardware gives
// for the same instruction as well as against the published peak.
#include "mpcg_internal.h"

namespace mpcg {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Eight independent accumulators per wavefront: each recurs only every
// eight instructions, more than the instruction's latency in passes.
__global__ __launch_bounds__(256) void mfma_i8_probe(int iters, int* sink) {
  const int t = (int)threadIdx.x;
  const v4i a = {t, 3, 5, 7}, b = {11, t, 13, 17};
  v4i c0 = {0, 0, 0, t}, c1 = {1, 0, 0, t}, c2 = {2, 0, 0, t}, c3 = {3, 0, 0, t}, c4 = {4, 0, 0, t},
      c5 = {5, 0, 0, t}, c6 = {6, 0, 0, t}, c7 = {7, 0, 0, t};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c7, 0, 0, 0);
  }
  const v4i s = c0 ^ c1 ^ c2 ^ c3 ^ c4 ^ c5 ^ c6 ^ c7;
  if (t == 0 && blockIdx.x == 0) sink[0] = s[0] ^ s[3];  // keeps every product live
}

__global__ __launch_bounds__(256) void mfma_f64_probe(int iters, int* sink) {
  const int t = (int)threadIdx.x;
  const double a = 1.0 + t * 0x1p-20, b = 1.0 - t * 0x1p-21;
  v4d c0 = {0.0, 0.0, 0.0, (double)t}, c1 = {1.0, 0.0, 0.0, (double)t}, c2 = {2.0, 0.0, 0.0, (double)t},
      c3 = {3.0, 0.0, 0.0, (double)t}, c4 = {4.0, 0.0, 0.0, (double)t}, c5 = {5.0, 0.0, 0.0, (double)t},
      c6 = {6.0, 0.0, 0.0, (double)t}, c7 = {7.0, 0.0, 0.0, (double)t};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c7, 0, 0, 0);
  }
  const v4d s = c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7;
  if (t == 0 && blockIdx.x == 0) sink[0] = (int)(s[0] + s[3] != 0.0);
}

}  // namespace

hipError_t launch_mfma_probe(int kind, int blocks, int iters, int* sink, hipStream_t stream) {
  if (kind == 0)
    mfma_i8_probe<<<dim3(blocks), dim3(256), 0, stream>>>(iters, sink);
  else
    mfma_f64_probe<<<dim3(blocks), dim3(256), 0, stream>>>(iters, sink);
  return hipGetLastError();
}

}  // namespace mpcg
