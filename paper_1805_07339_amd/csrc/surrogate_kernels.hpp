// BF16 MFMA kernels of the learned flow surrogate (gfx950): implicit-GEMM
// 3x3 convolutions (forward, input gradient, weight gradient with a
// deterministic split over pixels), the network input, the bilinear flow
// upsampling and its adjoint inside the Charbonnier loss, Adam, and the
// brightness-constancy residual gate.
//
// Layout: activations are NHWC bf16 (channels innermost), so the K
// dimension of every convolution GEMM is (tap, channel) with channels
// contiguous and one 16-byte load feeds one MFMA operand fragment.
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l holds A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] (j = 0..7) and receives
// D[4 (l / 16) + i][l % 16] (i = 0..3).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace scn {
namespace sg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint16_t bf16_t;

// Network shape (conv1..conv6), see the layer table in the header.
constexpr int kLayers = 6;
struct LayerDef {
  int ci, co, stride, up, relu;
};
constexpr LayerDef kNet[kLayers] = {{2, 32, 1, 0, 1},  {32, 64, 2, 0, 1}, {64, 96, 2, 0, 1},
                                    {96, 64, 1, 1, 1}, {64, 32, 1, 1, 1}, {32, 2, 1, 0, 0}};
constexpr int cpad(int c) { return (c + 15) / 16 * 16; }

// Parameter offsets (floats) in the master vector: per layer w[co][ci][3][3] then b[co].
constexpr int param_w_off(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += kNet[i].co * kNet[i].ci * 9 + kNet[i].co;
  return o;
}
constexpr int param_b_off(int l) { return param_w_off(l) + kNet[l].co * kNet[l].ci * 9; }
constexpr int kParams = param_w_off(kLayers);
static_assert(kParams == 148898, "parameter count");

// Packed network blob (device): per layer, forward weights bf16, transposed
// weights bf16 for the input gradient, bias f32.
//   forward:  [9][cpad(co)][ci] bf16, or for ci == 2 [cpad(co)][32] with k = 2 tap + ci
//   transpose: [9][ci][co] bf16, or for co == 2 [cpad(ci)][32] with k = 2 tap + co
constexpr int64_t fwd_elems(int l) {
  return kNet[l].ci == 2 ? (int64_t)cpad(kNet[l].co) * 32 : (int64_t)9 * cpad(kNet[l].co) * kNet[l].ci;
}
constexpr int64_t tr_elems(int l) {
  return kNet[l].co == 2 ? (int64_t)cpad(kNet[l].ci) * 32 : (int64_t)9 * kNet[l].ci * kNet[l].co;
}
constexpr int64_t align_elems(int64_t n) { return (n + 127) / 128 * 128; }
constexpr int64_t blob_fwd_off(int l) {
  int64_t o = 0;
  for (int i = 0; i < l; ++i) o += 2 * align_elems(fwd_elems(i)) + 2 * align_elems(tr_elems(i)) + 4 * align_elems(cpad(kNet[i].co));
  return o;
}
constexpr int64_t blob_tr_off(int l) { return blob_fwd_off(l) + 2 * align_elems(fwd_elems(l)); }
constexpr int64_t blob_bias_off(int l) { return blob_tr_off(l) + 2 * align_elems(tr_elems(l)); }
constexpr int64_t kBlobBytes = blob_fwd_off(kLayers);

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
// Global load at a base pointer plus a 32-bit byte offset (no per-lane
// 64-bit address arithmetic; the access is known to be global memory).
template <typename T>
__device__ __forceinline__ T ldg32(const T* base, uint32_t byte_off) {
  return *(const __attribute__((address_space(1))) T*)(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void stg32(T* base, uint32_t byte_off, T v) {
  *(__attribute__((address_space(1))) T*)(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Two floats to packed BF16 (a in the low half), round to nearest even: one
// v_cvt_pk_bf16_f32 on gfx950; equal to f2bf on finite inputs.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

}  // namespace sg
}  // namespace scn
