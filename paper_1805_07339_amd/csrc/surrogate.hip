// Learned flow surrogate for gfx950: BF16 MFMA implicit-GEMM convolutions
// (forward, input gradient, weight gradient), network input, flow
// upsampling, Charbonnier loss with its adjoint, Adam, and the residual
// gate.  Layouts and the MFMA lane mapping are described in
// surrogate_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "flow_plan.hpp"
#include "surrogate_kernels.hpp"

namespace scn {
namespace sg {

namespace {

struct CGeom {
  int32_t n;        // images (pairs) in the batch
  int32_t hi, wi;   // stored input size
  int32_t he, we;   // effective input size (2x the stored size for upsampled inputs)
  int32_t ho, wo;   // output size
};

__device__ __forceinline__ bf16x8 ld8(const bf16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x8 zero8() {
  const uint4 z = make_uint4(0, 0, 0, 0);
  return __builtin_bit_cast(bf16x8, z);
}
__device__ __forceinline__ bf16x8 pack8(const bf16_t (&v)[8]) {
  uint4 u;
  u.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
  u.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
  u.z = (uint32_t)v[4] | ((uint32_t)v[5] << 16);
  u.w = (uint32_t)v[6] | ((uint32_t)v[7] << 16);
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// Forward accumulators start at the bias (the MFMA's C operand), so the
// epilogue has no separate bias add.
__device__ __forceinline__ f32x4 bias4(const float* bias, int co) { return *reinterpret_cast<const f32x4*>(bias + co); }
// ReLU of two BF16 values packed in a dword: a BF16 is negative exactly when
// its 16-bit pattern is negative as int16, so a packed int16 max with 0 is
// the ReLU; ReLU commutes with rounding to BF16, so ReLU after packing
// equals packing after ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{0, 0}));
}

// ---------------------------------------------------------------------------
// forward: y[m][co] = act(bias[co] + sum_{tap, ci} W[tap][co][ci] x_e(m, tap)[ci])
// conv1 (2 input channels; the other layers use the LDS-tiled kernels): one
// wave computes 16*MR output pixels x all output channels.
template <int L, int MR>
__global__ void __launch_bounds__(256) k_conv_fwd(const bf16_t* __restrict__ x, const uint8_t* __restrict__ blob,
                                                  void* __restrict__ y, CGeom g) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, COP = cpad(CO), NB = COP / 16;
  static_assert(CI == 2, "two input channels: K = 18 fits one MFMA K block");
  constexpr bool UP = D.up != 0, RELU = D.relu != 0;
  const bf16_t* wf = reinterpret_cast<const bf16_t*>(blob + blob_fwd_off(L));
  const float* bias = reinterpret_cast<const float*>(blob + blob_bias_off(L));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t M = (int64_t)g.n * g.ho * g.wo;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wv) * (16 * MR);
  int pn[MR], poy[MR], pox[MR];
  bool pv[MR];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr) {
    const int64_t m = base + mr * 16 + r16;
    pv[mr] = m < M;
    const int64_t mm = pv[mr] ? m : 0;
    pox[mr] = (int)(mm % g.wo);
    const int64_t t = mm / g.wo;
    poy[mr] = (int)(t % g.ho);
    pn[mr] = (int)(t / g.ho);
  }
  f32x4 acc[MR][NB];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mr][nb] = bias4(bias, nb * 16 + 4 * kg);

  // K = 18 (9 taps x 2 channels) in one block of 32: lane group kg covers taps 4kg .. 4kg+3.
  bf16x8 a[MR];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr) {
    bf16_t v[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int tap = 4 * kg + j;
      uint32_t pair = 0;
      if (tap < 9) {
        const int iy = poy[mr] * S + tap / 3 - 1, ix = pox[mr] * S + tap % 3 - 1;
        if (pv[mr] && iy >= 0 && iy < g.he && ix >= 0 && ix < g.we) {
          const int sy = UP ? iy >> 1 : iy, sx = UP ? ix >> 1 : ix;
          pair = *reinterpret_cast<const uint32_t*>(x + (((int64_t)pn[mr] * g.hi + sy) * g.wi + sx) * 2);
        }
      }
      v[2 * j] = (bf16_t)(pair & 0xFFFFu);
      v[2 * j + 1] = (bf16_t)(pair >> 16);
    }
    a[mr] = pack8(v);
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const bf16x8 b = ld8(wf + (nb * 16 + r16) * 32 + kg * 8);
#pragma unroll
    for (int mr = 0; mr < MR; ++mr) acc[mr][nb] = mfma(b, a[mr], acc[mr][nb]);
  }
  // lane (r16, kg) holds channels nb*16 + 4kg .. +3 of pixel r16 of each block
#pragma unroll
  for (int mr = 0; mr < MR; ++mr) {
    const int64_t m = base + mr * 16 + r16;
    if (m >= M) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + 4 * kg;
      const f32x4 v = acc[mr][nb];  // bias included
      if constexpr (L == kLayers - 1) {
        if (co == 0) *reinterpret_cast<float2*>(reinterpret_cast<float*>(y) + m * CO) = make_float2(v[0], v[1]);
      } else {
        static_assert(L == kLayers - 1 || CO % 4 == 0, "epilogue stores 4 channels per lane");
        uint2 pk;
        pk.x = pack_bf16x2(v[0], v[1]);
        pk.y = pack_bf16x2(v[2], v[3]);
        if (RELU) {
          pk.x = relu_bf16x2(pk.x);
          pk.y = relu_bf16x2(pk.y);
        }
        *reinterpret_cast<uint2*>(reinterpret_cast<bf16_t*>(y) + m * CO + co) = pk;
      }
    }
  }
}

// Forward convolution with the input tile in LDS: a workgroup owns TOH x TOW
// output pixels of one image; the (TOH-1)S+3 x (TOW-1)S+3 effective input
// pixels it reads (zero outside the image, nearest-upsampled for x2 layers)
// are loaded once with 16-byte loads into LDS (channel stride padded by 8 to
// spread banks), and all nine taps read their fragments from there, so each
// input element crosses the memory hierarchy once per workgroup instead of
// nine times.  Each wave owns 16 * MR output pixels (MR pixel blocks of 16
// along a row) x all output channels.
//
// Latency: every thread issues all of its tile loads before the first LDS
// store, and the weight fragments of the next (tap row, channel block) step
// are requested while the current step's MFMAs run.  The MFMA takes the
// weights as its first operand, so a lane's accumulator holds four
// consecutive output channels of one pixel and the epilogue stores 8 bytes
// per lane.  BLDS stages the whole weight tensor in LDS as well.
// MFMA part of the LDS-tiled forward convolution, shared by the kernels that
// stage a tile: `tile` holds the layer's input tile (SH x SW stored pixels,
// channel stride tile_cp(L)), `wf` the forward weights [tap][co][ci] (LDS or
// global).  Each wave owns 16 * MR output pixels (MR pixel blocks of 16 along
// a row) x all output channels; the epilogue adds the bias, applies ReLU and
// stores 4 consecutive channels per lane.
// Weights staged in LDS keep the [tap][co][ci] layout with the 16-byte
// chunks of each row XOR-swizzled: a B fragment read touches 16 consecutive
// rows at one chunk, and with rows of 2 CI bytes several of those rows would
// start in the same bank (CI = 96: rows r and r + 4; CI = 64: every second
// row).  Chunk c of row r is stored at c ^ ((r >> SH) & MASK), where rows
// that repeat a bank offset (period P = 256 / gcd(256, 2 CI) rows) differ
// in r >> SH: the 16 rows of a read then hit 16 distinct 4-bank groups.
constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }
constexpr int log2_i(int v) { return v <= 1 ? 0 : 1 + log2_i(v / 2); }
// Channel stride of a staged input tile: 8 channels of padding, 16 for the
// last layer (32 input channels), whose tile reads run faster with it.
constexpr int tile_cp(int l) { return kNet[l].ci + (l == kLayers - 1 ? 16 : 8); }

template <int CI> struct WSwz {
  static constexpr int P = 256 / gcd_i(256, 2 * CI);
  static constexpr int SH = log2_i(P), MASK = 16 / P - 1;
  static_assert((P & (P - 1)) == 0 && (CI / 8) % (MASK + 1) == 0, "swizzle stays inside the row");
  // element offset of chunk c8 of row r
  static __device__ __forceinline__ int off(int r, int c8) { return r * CI + ((c8 ^ ((r >> SH) & MASK)) << 3); }
};

template <int L, int TOH, int TOW, int NWAVE, int SH, int SW, bool WLDS>
__device__ __forceinline__ void conv_tile_mma(const bf16_t* __restrict__ tile, const bf16_t* __restrict__ wf,
                                              const float* __restrict__ bias, void* __restrict__ y, const CGeom& g,
                                              int n, int oy0, int ox0) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, COP = cpad(CO), NB = COP / 16, NCB = CI / 32;
  constexpr bool UP = D.up != 0, RELU = D.relu != 0;
  constexpr int CP = tile_cp(L);
  constexpr int BPR = TOW / 16, NBLK = TOH * BPR, MR = NBLK / NWAVE;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const uint32_t blane = 2u * (uint32_t)(r16 * CI + kg * 8);  // lane's byte offset in a fragment row block
  auto bfrag = [&](int tap, int nb, int cb) -> bf16x8 {
    const bf16_t* base = wf + (tap * COP + nb * 16) * CI + cb * 32;  // wave-uniform
    if constexpr (WLDS) return ld8(wf + WSwz<CI>::off(tap * COP + nb * 16 + r16, cb * 4 + kg));
    else return ldg32(reinterpret_cast<const bf16x8*>(base), blane);
  };
  f32x4 acc[MR][NB];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mr][nb] = bias4(bias, nb * 16 + 4 * kg);
  if constexpr (S == 1 && UP) {
    // x2 nearest-upsampled input: effective index e reads stored index
    // (e + 1) >> 1, so the nine taps of a pixel touch only two stored rows
    // (R0 = ti(orow), R2 = ti(orow + 2); tap row 1 reads R0 for odd and R2
    // for even output rows) and two stored columns (C0 = ti(c), C2 = ti(c + 2);
    // tap column 1 reads C0 for odd and C2 for even output columns).  The
    // four distinct fragments of a (block, channel block) are read once: the
    // R0 pair at tap row 0, the R2 pair at tap row 1; the middle taps are
    // selects.  Same fragments and MFMA order as the general path below.
    constexpr int NST = 3 * NCB;  // steps: (ky, channel block)
    bf16x8 bq[2][3][NB];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bq[0][kx][nb] = bfrag(kx, nb, 0);
    auto ti = [](int e) { return (e + 1) >> 1; };  // effective -> stored tile index
    const bool odd_col = (r16 & 1) != 0;           // c0 is a multiple of 16
    bf16x8 f0[NCB][MR][2], f2[NCB][MR][2];          // [cb][mr][C0, C2] of rows R0, R2
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int ky = st / NCB, cb = st % NCB, cur = st & 1;
      if (st + 1 < NST) {
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) bq[cur ^ 1][kx][nb] = bfrag(((st + 1) / NCB) * 3 + kx, nb, (st + 1) % NCB);
      }
      bf16x8 a0[MR], a1[MR], a2[MR];
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) {
        const int blk = wv * MR + mr;
        const int orow = blk / BPR, c0 = (blk % BPR) * 16;
        if (ky < 2) {  // ky = 0 reads the R0 pair, ky = 1 the R2 pair
          const int R = ti(orow + 2 * ky);
          const bf16_t* rowp = tile + (R * SW) * CP + cb * 32 + kg * 8;
          bf16x8(&f)[2] = ky == 0 ? f0[cb][mr] : f2[cb][mr];
          f[0] = ld8(rowp + ti(c0 + r16) * CP);
          f[1] = ld8(rowp + ti(c0 + r16 + 2) * CP);
        }
        const bool use_r0 = ky == 0 || (ky == 1 && (orow & 1));
        const bf16x8 g0 = use_r0 ? f0[cb][mr][0] : f2[cb][mr][0];
        const bf16x8 g2 = use_r0 ? f0[cb][mr][1] : f2[cb][mr][1];
        a0[mr] = g0;
        a2[mr] = g2;
        a1[mr] = odd_col ? g0 : g2;
      }
#pragma unroll
      for (int kx = 0; kx < 3; ++kx)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int mr = 0; mr < MR; ++mr)
            acc[mr][nb] = mfma(bq[cur][kx][nb], kx == 0 ? a0[mr] : (kx == 1 ? a1[mr] : a2[mr]), acc[mr][nb]);
    }
  } else if constexpr (S == 1) {
    // Stride 1: the three taps of a tap row read consecutive pixels of one
    // tile row (one 16-byte LDS read per tap and pixel block).
    constexpr int NST = 3 * NCB;  // steps: (ky, channel block)
    bf16x8 bq[2][3][NB];
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) bq[0][kx][nb] = bfrag(kx, nb, 0);
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int ky = st / NCB, cb = st % NCB, cur = st & 1;
      if (st + 1 < NST) {
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) bq[cur ^ 1][kx][nb] = bfrag(((st + 1) / NCB) * 3 + kx, nb, (st + 1) % NCB);
      }
      bf16x8 a0[MR], a1[MR], a2[MR];
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) {
        const int blk = wv * MR + mr;
        const int orow = blk / BPR, c0 = (blk % BPR) * 16;
        auto ti = [](int e) { return UP ? (e + 1) >> 1 : e; };  // effective -> stored tile index
        const bf16_t* rowp = tile + (ti(orow + ky) * SW) * CP + cb * 32 + kg * 8;
        a0[mr] = ld8(rowp + ti(c0 + r16) * CP);
        a1[mr] = ld8(rowp + ti(c0 + r16 + 1) * CP);
        a2[mr] = ld8(rowp + ti(c0 + r16 + 2) * CP);
      }
#pragma unroll
      for (int kx = 0; kx < 3; ++kx)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int mr = 0; mr < MR; ++mr)
            acc[mr][nb] = mfma(bq[cur][kx][nb], kx == 0 ? a0[mr] : (kx == 1 ? a1[mr] : a2[mr]), acc[mr][nb]);
    }
  } else {
    constexpr int NST = 9 * NCB;  // steps: (tap, channel block)
    bf16x8 bq[2][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) bq[0][nb] = bfrag(0, nb, 0);
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int tap = st / NCB, cb = st % NCB, cur = st & 1;
      const int ky = tap / 3, kx = tap % 3;
      if (st + 1 < NST) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bq[cur ^ 1][nb] = bfrag((st + 1) / NCB, nb, (st + 1) % NCB);
      }
      bf16x8 a[MR];
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) {
        const int blk = wv * MR + mr;
        const int orow = blk / BPR, ocol = (blk % BPR) * 16 + r16;
        a[mr] = ld8(tile + ((orow * S + ky) * SW + ocol * S + kx) * CP + cb * 32 + kg * 8);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mr = 0; mr < MR; ++mr) acc[mr][nb] = mfma(bq[cur][nb], a[mr], acc[mr][nb]);
    }
  }
  // lane (r16, kg) holds channels nb*16 + 4kg .. +3 of pixel r16 of each block
  constexpr int OBYTES = L == kLayers - 1 ? 4 : 2;  // FP32 flow or BF16 activation
  char* yimg = reinterpret_cast<char*>(y) + (int64_t)n * g.ho * g.wo * CO * OBYTES;  // wave-uniform
#pragma unroll
  for (int mr = 0; mr < MR; ++mr) {
    const int blk = wv * MR + mr;
    const int oy = oy0 + blk / BPR, ox = ox0 + (blk % BPR) * 16 + r16;
    if (oy >= g.ho || ox >= g.wo) continue;
    const uint32_t mo = (uint32_t)(oy * g.wo + ox) * (uint32_t)(CO * OBYTES);  // pixel's byte offset in the image
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int co = nb * 16 + 4 * kg;
      const f32x4 v = acc[mr][nb];  // bias included
      if constexpr (L == kLayers - 1) {
        static_assert(CO == 2 && !RELU, "last layer writes (u, v)");
        if (co == 0) stg32(reinterpret_cast<f32x2_t*>(yimg), mo, f32x2_t{v[0], v[1]});
      } else {
        uint2 pk;
        pk.x = pack_bf16x2(v[0], v[1]);
        pk.y = pack_bf16x2(v[2], v[3]);
        if (RELU) {
          pk.x = relu_bf16x2(pk.x);
          pk.y = relu_bf16x2(pk.y);
        }
        typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
        stg32(reinterpret_cast<u32x2_t*>(yimg), mo + 2u * (uint32_t)co, u32x2_t{pk.x, pk.y});
      }
    }
  }
}


template <int L, int TOH, int TOW, int NWAVE, bool BLDS>
__global__ void __launch_bounds__(64 * NWAVE) k_conv_fwd_lds(const bf16_t* __restrict__ x,
                                                             const uint8_t* __restrict__ blob, void* __restrict__ y,
                                                             CGeom g, int32_t tiles_x, int32_t tiles_per_img) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, COP = cpad(CO), NB = COP / 16, NCB = CI / 32;
  constexpr bool UP = D.up != 0, RELU = D.relu != 0;
  constexpr int IH = (TOH - 1) * S + 3, IW = (TOW - 1) * S + 3, CP = tile_cp(L);
  constexpr int BPR = TOW / 16, NBLK = TOH * BPR, MR = NBLK / NWAVE;
  constexpr int NT = 64 * NWAVE;
  constexpr int WELEMS = BLDS ? 9 * COP * CI : 8;
  static_assert(CI % 32 == 0 && TOW % 16 == 0 && NBLK % NWAVE == 0, "tile shape");
  static_assert(CO % 4 == 0 || L == kLayers - 1, "epilogue stores 4 channels per lane");
  // x2-upsampled layers keep the source-resolution tile: effective tile
  // index e (rows or columns) maps to source index (e + 1) / 2 because the
  // tile origin oy0 - 1, ox0 - 1 is odd (TOH, TOW even), so the tile is a
  // quarter of the effective one.
  static_assert(!UP || (S == 1 && TOH % 2 == 0 && TOW % 2 == 0), "upsampled tile shape");
  constexpr int SH = UP ? IH / 2 + 1 : IH, SW = UP ? IW / 2 + 1 : IW;
  __shared__ __attribute__((aligned(16))) bf16_t tile[SH * SW * CP];
  __shared__ __attribute__((aligned(16))) bf16_t wlds[WELEMS];
  const float* bias = reinterpret_cast<const float*>(blob + blob_bias_off(L));
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int n = blk / tiles_per_img;
  const int t = blk % tiles_per_img;
  const int oy0 = (t / tiles_x) * TOH, ox0 = (t % tiles_x) * TOW;
  const int iy0 = oy0 * S - 1, ix0 = ox0 * S - 1;

  // ---- stage: all global loads first, then all LDS stores
  constexpr int NW8 = BLDS ? WELEMS / 8 : 0, WIT = (NW8 + NT - 1) / NT;
  constexpr int NE = SH * SW * (CI / 8), IT = (NE + NT - 1) / NT;
  const uint4* wsrc = reinterpret_cast<const uint4*>(blob + blob_fwd_off(L));
  uint4 wreg[WIT > 0 ? WIT : 1];
#pragma unroll
  for (int i = 0; i < WIT; ++i) wreg[i] = wsrc[min(tid + i * NT, NW8 - 1)];
  uint4 treg[IT];
  const bf16_t* ximg = x + (int64_t)n * g.hi * g.wi * CI;  // this image's input (wave-uniform)
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = min(tid + i * NT, NE - 1);
    const int ch = e % (CI / 8), p = e / (CI / 8);
    // stored coordinates (source resolution for upsampled layers)
    const int yy = (UP ? (iy0 >> 1) : iy0) + p / SW, xx = (UP ? (ix0 >> 1) : ix0) + p % SW;
    const bool ok = yy >= 0 && yy < g.hi && xx >= 0 && xx < g.wi;
    const int sy = ok ? yy : 0, sx = ok ? xx : 0;
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    const u32x4_t v = ldg32(reinterpret_cast<const u32x4_t*>(ximg), 2u * (uint32_t)((sy * g.wi + sx) * CI + ch * 8));
    treg[i] = ok ? make_uint4(v.x, v.y, v.z, v.w) : make_uint4(0, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < WIT; ++i) {
    const int c = tid + i * NT;  // 16-byte chunk c8 of weight row r
    if (c < NW8) *reinterpret_cast<uint4*>(wlds + WSwz<CI>::off(c / (CI / 8), c % (CI / 8))) = wreg[i];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int e = tid + i * NT;
    if (e < NE) *reinterpret_cast<uint4*>(tile + (e / (CI / 8)) * CP + (e % (CI / 8)) * 8) = treg[i];
  }
  __syncthreads();

  const bf16_t* wf = BLDS ? wlds : reinterpret_cast<const bf16_t*>(blob + blob_fwd_off(L));
  conv_tile_mma<L, TOH, TOW, NWAVE, SH, SW, BLDS>(tile, wf, bias, y, g, n, oy0, ox0);
}

// Persistent form of the LDS-tiled forward convolution for layers whose
// weights live in LDS: a workgroup stages the weights once and then walks
// output tiles t, t + gridDim.x, ...  The input tile is double-buffered: the global loads of the next tile are issued before
// the MFMAs of the current one and written to the other LDS buffer after
// them, so staging overlaps compute, and the weight tensor crosses the
// memory hierarchy once per workgroup instead of once per tile.
template <int L, int TOH, int TOW, int NWAVE, int WPE>
__global__ void __launch_bounds__(64 * NWAVE, WPE) k_conv_fwd_pers(const bf16_t* __restrict__ x,
                                                              const uint8_t* __restrict__ blob, void* __restrict__ y,
                                                              CGeom g, int32_t tiles_x, int32_t tiles_per_img,
                                                              int32_t n_tiles) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, COP = cpad(CO);
  constexpr bool UP = D.up != 0;
  constexpr int IH = (TOH - 1) * S + 3, IW = (TOW - 1) * S + 3, CP = tile_cp(L);
  constexpr int NT = 64 * NWAVE;
  constexpr int WELEMS = 9 * COP * CI;
  static_assert(CI % 32 == 0 && TOW % 16 == 0 && (TOH * TOW / 16) % NWAVE == 0, "tile shape");
  static_assert(!UP || (S == 1 && TOH % 2 == 0 && TOW % 2 == 0), "upsampled tile shape");
  constexpr int SH = UP ? IH / 2 + 1 : IH, SW = UP ? IW / 2 + 1 : IW;
  constexpr int TILE = SH * SW * CP;
  __shared__ __attribute__((aligned(16))) bf16_t tile[2 * TILE];
  __shared__ __attribute__((aligned(16))) bf16_t wlds[WELEMS];
  const float* bias = reinterpret_cast<const float*>(blob + blob_bias_off(L));
  const int tid = threadIdx.x;
  constexpr int NW8 = WELEMS / 8, WIT = (NW8 + NT - 1) / NT;
  constexpr int NE = SH * SW * (CI / 8), IT = (NE + NT - 1) / NT;
  typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
  uint4 treg[IT];
  // global loads of tile t's input into treg (zero outside the image)
  auto load_tile = [&](int t) {
    const int n = t / tiles_per_img, r = t % tiles_per_img;
    const int iy0 = (r / tiles_x) * TOH * S - 1, ix0 = (r % tiles_x) * TOW * S - 1;
    const bf16_t* ximg = x + (int64_t)n * g.hi * g.wi * CI;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = min(tid + i * NT, NE - 1);
      const int ch = e % (CI / 8), p = e / (CI / 8);
      const int yy = (UP ? (iy0 >> 1) : iy0) + p / SW, xx = (UP ? (ix0 >> 1) : ix0) + p % SW;
      const bool ok = yy >= 0 && yy < g.hi && xx >= 0 && xx < g.wi;
      const int sy = ok ? yy : 0, sx = ok ? xx : 0;
      const u32x4_t v = ldg32(reinterpret_cast<const u32x4_t*>(ximg), 2u * (uint32_t)((sy * g.wi + sx) * CI + ch * 8));
      treg[i] = ok ? make_uint4(v.x, v.y, v.z, v.w) : make_uint4(0, 0, 0, 0);
    }
  };
  auto store_tile = [&](bf16_t* buf) {
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = tid + i * NT;
      if (e < NE) *reinterpret_cast<uint4*>(buf + (e / (CI / 8)) * CP + (e % (CI / 8)) * 8) = treg[i];
    }
  };
  // round k covers tiles k*G .. k*G + G - 1 (G = gridDim.x), spread so that
  // each XCD takes a contiguous part of them
  int t = xcd_block(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return;  // uniform over the workgroup, before any barrier
  {
    const uint4* wsrc = reinterpret_cast<const uint4*>(blob + blob_fwd_off(L));
    uint4 wreg[WIT];
#pragma unroll
    for (int i = 0; i < WIT; ++i) wreg[i] = wsrc[min(tid + i * NT, NW8 - 1)];
    load_tile(t);
#pragma unroll
    for (int i = 0; i < WIT; ++i) {
      const int c = tid + i * NT;  // 16-byte chunk c8 of weight row r
      if (c < NW8) *reinterpret_cast<uint4*>(wlds + WSwz<CI>::off(c / (CI / 8), c % (CI / 8))) = wreg[i];
    }
    store_tile(tile);
  }
  __syncthreads();
  for (int buf = 0; t < n_tiles; t += gridDim.x, buf ^= 1) {
    const int tn = t + gridDim.x;
    if (tn < n_tiles) load_tile(tn);  // in flight during this tile's MFMAs
    const int n = t / tiles_per_img, r = t % tiles_per_img;
    conv_tile_mma<L, TOH, TOW, NWAVE, SH, SW, true>(tile + buf * TILE, wlds, bias, y, g, n, (r / tiles_x) * TOH,
                                                    (r % tiles_x) * TOW);
    if (tn < n_tiles) store_tile(tile + (buf ^ 1) * TILE);  // that buffer was last read before the previous barrier
    __syncthreads();
  }
}

// Stride-2 layer (conv3: 64 -> 96, its weights are 110 KB) as a persistent
// kernel: the workgroup stages the weights once in LDS (rows padded to CI + 8
// channels, so the 16 rows a fragment read touches fall in distinct banks)
// and then each wave walks tasks of one output row x 16 MR columns on its
// own: no barrier after the staging.  A fragments come straight from global
// memory (L2; zero outside the image), requested two (tap, channel-block)
// steps ahead of their MFMAs; the six B fragments of a step are LDS reads
// shared by the MR pixel blocks.  Same fragments, MFMA order and epilogue as
// the tiled kernel, so the output is bitwise the same.
template <int L, int MR>
__global__ void __launch_bounds__(256) k_conv_s2_pers(const bf16_t* __restrict__ x, const uint8_t* __restrict__ blob,
                                                      bf16_t* __restrict__ y, CGeom g, int32_t tasks_x,
                                                      int32_t n_tasks) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, COP = cpad(CO), NB = COP / 16, NCB = CI / 32, WP = CI + 8;
  constexpr bool RELU = D.relu != 0;
  static_assert(D.stride == 2 && !D.up && CO % 16 == 0 && CI % 32 == 0, "stride-2 layer");
  constexpr int NST = 9 * NCB, DEPTH = 3;
  __shared__ __attribute__((aligned(16))) bf16_t wlds[9 * COP * WP];
  const int tid = threadIdx.x, lane = tid & 63, r16 = lane & 15, kg = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  {
    constexpr int NCH = 9 * COP * CI / 8, IT = (NCH + 255) / 256;  // 16-byte chunks
    const uint4* wsrc = reinterpret_cast<const uint4*>(blob + blob_fwd_off(L));
    uint4 reg[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) reg[i] = wsrc[min(tid + i * 256, NCH - 1)];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int c = tid + i * 256;
      if (c < NCH) *reinterpret_cast<uint4*>(wlds + (c / (CI / 8)) * WP + (c % (CI / 8)) * 8) = reg[i];
    }
  }
  __syncthreads();
  const float* bias = reinterpret_cast<const float*>(blob + blob_bias_off(L));
  const uint32_t img_bytes = (uint32_t)g.hi * (uint32_t)g.wi * (uint32_t)(CI * 2);
  const int32_t per_img = g.ho * tasks_x;
  const int32_t nw = (int32_t)gridDim.x * 4;
  for (int32_t task = (int32_t)xcd_block(blockIdx.x, gridDim.x) * 4 + wv; task < n_tasks; task += nw) {
    const int32_t n = task / per_img, rem = task % per_img;
    const int32_t oy = rem / tasks_x, ox0 = (rem % tasks_x) * (16 * MR);
    // The image as a buffer resource: an offset past its end reads zeros,
    // which is the zero padding (no branch around the loads).
    const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(reinterpret_cast<const char*>(x) + (size_t)n * img_bytes), (short)0, (int)img_bytes, 0x00020000);
    // A fragment of block mr at step st: input pixel (2 oy + ky - 1, 2 ox + kx - 1), channels cb*32 + kg*8 ..
    auto load_a = [&](int st, bf16x8 (&a)[MR]) {
      const int tap = st / NCB, cb = st % NCB, ky = tap / 3, kx = tap % 3;
      const int32_t iy = 2 * oy + ky - 1;
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) {
        const int32_t ix = 2 * (ox0 + 16 * mr + r16) + kx - 1;
        const bool ok = iy >= 0 && iy < g.hi && ix >= 0 && ix < g.wi;
        const uint32_t off = ok ? ((uint32_t)(iy * g.wi + ix) * CI + cb * 32 + kg * 8) * 2u : 0x80000000u;
        a[mr] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
      }
    };
    f32x4 acc[MR][NB];
#pragma unroll
    for (int mr = 0; mr < MR; ++mr)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mr][nb] = bias4(bias, nb * 16 + 4 * kg);
    // A ring of DEPTH steps; the step loop runs DEPTH steps per iteration so
    // that ring slots stay compile-time registers, and is not unrolled
    // further (unrolled, the loads of all steps are hoisted and spill); the
    // last DEPTH steps, which request nothing ahead, are peeled.
    static_assert(NST % DEPTH == 0 && NST > DEPTH, "step count");
    bf16x8 abuf[DEPTH][MR];
    auto mma_step = [&](int st, const bf16x8 (&a)[MR]) {
      const int tap = st / NCB, cb = st % NCB;
      bf16x8 b[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) b[nb] = ld8(wlds + (tap * COP + nb * 16 + r16) * WP + cb * 32 + kg * 8);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mr = 0; mr < MR; ++mr) acc[mr][nb] = mfma(b[nb], a[mr], acc[mr][nb]);
    };
#pragma unroll
    for (int st = 0; st < DEPTH - 1; ++st) load_a(st, abuf[st]);
#pragma unroll 1
    for (int sg = 0; sg < NST - DEPTH; sg += DEPTH) {
#pragma unroll
      for (int j = 0; j < DEPTH; ++j) {
        load_a(sg + j + DEPTH - 1, abuf[(j + DEPTH - 1) % DEPTH]);
        mma_step(sg + j, abuf[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < DEPTH; ++j) {
      if (j == 0) load_a(NST - 1, abuf[DEPTH - 1]);
      mma_step(NST - DEPTH + j, abuf[j]);
    }
    // epilogue: lane (r16, kg) holds channels nb*16 + 4kg .. +3 of pixel r16 of each block
    char* yrow = reinterpret_cast<char*>(y) + ((size_t)n * g.ho + oy) * (size_t)g.wo * (CO * 2);  // wave-uniform
#pragma unroll
    for (int mr = 0; mr < MR; ++mr) {
      const int32_t ox = ox0 + 16 * mr + r16;
      if (ox >= g.wo) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int co = nb * 16 + 4 * kg;
        const f32x4 v = acc[mr][nb];  // bias included
        uint32_t p0 = pack_bf16x2(v[0], v[1]), p1 = pack_bf16x2(v[2], v[3]);
        if (RELU) {
          p0 = relu_bf16x2(p0);
          p1 = relu_bf16x2(p1);
        }
        typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
        stg32(reinterpret_cast<u32x2_t*>(yrow), (uint32_t)(ox * CO + co) * 2u, u32x2_t{p0, p1});
      }
    }
  }
}

// Inference: conv1 (2 -> 32, stride 1) and conv2 (32 -> 64, stride 2) in one
// persistent kernel without an LDS tile of conv1 outputs.  A wave owns a
// strip of 64 conv2 output columns (4 blocks of 16 pixels) and a band of
// output rows and streams down it.  Per output row and conv2 tap, the conv1
// outputs the tap reads (each block's 16 pixels, two apart) are computed
// straight into conv2's fragment layout: conv1's weight rows are taken in the
// order 0-3, 8-11, 16-19, 24-27 for the first 16-row MFMA block and 4-7,
// 12-15, 20-23, 28-31 for the second, so that lane (r16, kg) ends with
// channels 8kg .. 8kg + 7 of its pixel -- the eight BF16 values conv2's
// fragment needs -- after the same bias, rounding and ReLU as the
// standalone conv1 (zero outside the image: conv2's padding).  A conv1
// output is recomputed by each conv2 tap that reads it (2.25 on average):
// the price of no LDS round trip and no barrier.  The network input (2x2
// luma means of both frames in BF16, the arithmetic of k_net_input) of the
// strip's rows sits in a per-wave ring of 8 rows in LDS; the two rows the
// next output row needs are loaded during the current row's MFMAs.  conv2's
// weights are staged in LDS once per workgroup.  Every output sees the MFMA
// sequence of the unfused layers (conv1: one K block; conv2: taps in order,
// one 32-channel block), so the results are bitwise theirs.
constexpr int kC12sCols = 64;                      // conv2 output columns computed per strip (4 blocks)
constexpr int kC12sStep = 62;                      // of which stored: strips overlap by 2 columns
constexpr int kC12sRing = 8;                       // network-input rows per wave ring
constexpr int kC12sRW = 2 * kC12sCols + 4;         // ring row stride (2 * 64 + 3 columns read)
template <int NWAVE, int BAND>
__global__ void __launch_bounds__(64 * NWAVE) k_conv12s(const FrameDesc* __restrict__ frames,
                                                         const PairDesc* __restrict__ pairs,
                                                         const uint8_t* __restrict__ blob, bf16_t* __restrict__ y,
                                                         CGeom g1, CGeom g2, int32_t strips, int32_t bands,
                                                         int64_t units) {
  static_assert(kNet[0].ci == 2 && kNet[0].co == 32 && kNet[1].ci == 32 && kNet[1].co == 64 &&
                kNet[1].stride == 2, "layer shapes");
  constexpr int NT = 64 * NWAVE, W2 = 9 * 64 * 32, NCOL = 2 * kC12sStep + 3;
  static_assert(NCOL <= 128, "one pair of network-input columns per lane");
  // [wave][row slot][column]: two bf16 channels; slot kC12sRing stays zero
  // (the reads of conv1's padded K elements, taps 9 .. 11, point there)
  __shared__ uint32_t ring[NWAVE][kC12sRing + 1][kC12sRW];
  __shared__ __attribute__((aligned(16))) bf16_t w2[W2];  // conv2 weights [tap][co][ci], swizzled rows
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  {
    const uint4* wsrc = reinterpret_cast<const uint4*>(blob + blob_fwd_off(1));
    for (int c = tid; c < W2 / 8; c += NT) *reinterpret_cast<uint4*>(w2 + WSwz<32>::off(c / 4, c % 4)) = wsrc[c];
  }
  for (int c = lane; c < kC12sRW; c += 64) ring[wv][kC12sRing][c] = 0u;
  __syncthreads();  // the only barrier: waves are independent from here on
  const bf16_t* wf1 = reinterpret_cast<const bf16_t*>(blob + blob_fwd_off(0));
  const float* b1 = reinterpret_cast<const float*>(blob + blob_bias_off(0));
  const float* b2 = reinterpret_cast<const float*>(blob + blob_bias_off(1));
  // conv1 fragments in the permuted row order, and their biases
  bf16x8 bw1[2];
  f32x4 bv1[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    bw1[j] = ld8(wf1 + (8 * (r16 >> 2) + 4 * j + (r16 & 3)) * 32 + kg * 8);
    bv1[j] = bias4(b1, 8 * kg + 4 * j);
  }
  // lane group kg covers conv1's K elements 8kg .. 8kg+7 = taps 4kg .. 4kg+3
  // of the 3x3 window, two channels each (taps >= 9 are zero)
  int tdy[4], cbase[4];
  bool tok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int tap = 4 * kg + j;
    tok[j] = tap < 9;
    tdy[j] = tok[j] ? tap / 3 : 0;
    cbase[j] = 2 * r16 + (tok[j] ? tap % 3 : 0);  // ring column of the tap for block 0, kx = 0
  }
  uint32_t(&rg)[kC12sRing + 1][kC12sRW] = ring[wv];
  const uint32_t* rflat = &ring[wv][0][0];
  const int64_t per_pair = (int64_t)bands * strips;
  for (int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NWAVE + wv; unit < units;
       unit += (int64_t)gridDim.x * NWAVE) {
    const int n = (int)(unit / per_pair);
    const int rem = (int)(unit % per_pair);
    const int band = rem / strips, sx = rem % strips;
    const int ox0 = sx * kC12sStep, oy_a = band * BAND, oy_b = min(g2.ho, oy_a + BAND);
    const int xb = 2 * ox0 - 2;                                      // network-input column of ring column 0
    const PairDesc pd = pairs[n];
    const FrameDesc fa = frames[pd.f1], fb = frames[pd.f2];
    const uint32_t pa = (uint32_t)fa.pitch, pbp = (uint32_t)fb.pitch;
    // network-input row yy of the strip: lane l takes columns 2l, 2l + 1 (one
    // 4-byte load per luma row and frame covers both pixels' 2x2 blocks);
    // then the BF16 pairs go into the ring (the arithmetic of k_net_input;
    // zero outside the image).  Ring columns NCOL .. 130, read only for the
    // two computed outputs past kC12sStep, which are not stored, keep stale
    // values.
    auto load_row = [&](int yy, uint32_t (&lw)[4]) {
      const int c = 2 * lane, xx = xb + c;
      const bool ok = yy >= 0 && yy < g1.hi && xx >= 0 && xx + 1 < g1.wi;  // both pixels inside
      const uint32_t ry = 2u * (uint32_t)(yy >= 0 && yy < g1.hi ? yy : 0);
      const uint32_t rx = 2u * (uint32_t)(ok ? xx : 0);
      lw[0] = ldg32(reinterpret_cast<const uint32_t*>(fa.y), ry * pa + rx);
      lw[1] = ldg32(reinterpret_cast<const uint32_t*>(fa.y), (ry + 1) * pa + rx);
      lw[2] = ldg32(reinterpret_cast<const uint32_t*>(fb.y), ry * pbp + rx);
      lw[3] = ldg32(reinterpret_cast<const uint32_t*>(fb.y), (ry + 1) * pbp + rx);
    };
    auto store_row = [&](int yy, const uint32_t (&lw)[4]) {
      const bool yok = yy >= 0 && yy < g1.hi;
#pragma unroll
      for (int h = 0; h < 2; ++h) {  // pixel 2l + h: bytes 2h, 2h + 1 of each loaded word
        const int c = 2 * lane + h, xx = xb + c;
        const bool ok = yok && xx >= 0 && xx < g1.wi;
        const int s1 = (int)(((lw[0] >> (16 * h)) & 0xFFu) + ((lw[0] >> (16 * h + 8)) & 0xFFu) +
                             ((lw[1] >> (16 * h)) & 0xFFu) + ((lw[1] >> (16 * h + 8)) & 0xFFu));
        const int s2 = (int)(((lw[2] >> (16 * h)) & 0xFFu) + ((lw[2] >> (16 * h + 8)) & 0xFFu) +
                             ((lw[3] >> (16 * h)) & 0xFFu) + ((lw[3] >> (16 * h + 8)) & 0xFFu));
        const uint32_t v = pack_bf16x2((float)(((s1 + 2) >> 2) - 128) * (1.f / 64.f),
                                       (float)(((s2 + 2) >> 2) - 128) * (1.f / 64.f));
        if (c < NCOL) rg[yy & (kC12sRing - 1)][c] = ok ? v : 0u;
      }
    };
    for (int r = 0; r < 5; r += 2) {  // the band's first five rows, two at a time
      uint32_t lw[2][4];
      load_row(2 * oy_a - 2 + r, lw[0]);
      if (r + 1 < 5) load_row(2 * oy_a - 1 + r, lw[1]);
      store_row(2 * oy_a - 2 + r, lw[0]);
      if (r + 1 < 5) store_row(2 * oy_a - 1 + r, lw[1]);
    }
    // strips at the left or right image border hold conv1 columns outside
    // the image, and output row 0 reads conv1 row -1: those rows take the
    // path that zeroes such conv1 outputs (conv2's padding)
    const bool col_edge = xb + 1 < 0 || xb + 1 + 2 * kC12sCols + 1 >= g1.wo;
    for (int oy = oy_a; oy < oy_b; ++oy) {
      // the two network-input rows of the next output row, in flight during this row's MFMAs
      uint32_t nx[2][4];
      load_row(2 * oy + 3, nx[0]);
      load_row(2 * oy + 4, nx[1]);
      f32x4 acc[4][4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const f32x4 bias = bias4(b2, nb * 16 + 4 * kg);
#pragma unroll
        for (int mr = 0; mr < 4; ++mr) acc[mr][nb] = bias;
      }
      // word offsets of tap j's ring row for tap row ky of conv2 (the zero row
      // for conv1's padded K elements); block mr and tap column kx add
      // 32 mr + kx, a constant of the read instruction
      int roff[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
          roff[j][ky] = tok[j] ? ((2 * oy - 2 + ky + tdy[j]) & (kC12sRing - 1)) * kC12sRW + cbase[j]
                               : kC12sRing * kC12sRW;
      auto ring_a = [&](int t, int mr) {  // conv1 fragment of block mr for conv2 tap t
        const int ky = t / 3, kx = t % 3;
        uint4 pw;
        pw.x = rflat[roff[0][ky] + 32 * mr + kx];
        pw.y = rflat[roff[1][ky] + 32 * mr + kx];
        pw.z = rflat[roff[2][ky] + 32 * mr + kx];
        pw.w = rflat[roff[3][ky] + 32 * mr + kx];
        return pw;
      };
      auto taps = [&](auto edge) {
        constexpr bool EDGE = decltype(edge)::value;
        // the ring reads of tap t + 1 are issued before tap t's arithmetic
        uint4 pw[2][4];
#pragma unroll
        for (int mr = 0; mr < 4; ++mr) pw[0][mr] = ring_a(0, mr);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int ky = t / 3, kx = t % 3, cur = t & 1;
          bf16x8 bq[4];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) bq[nb] = ld8(w2 + WSwz<32>::off(t * 64 + nb * 16 + r16, kg));
          if (t + 1 < 9) {
#pragma unroll
            for (int mr = 0; mr < 4; ++mr) pw[cur ^ 1][mr] = ring_a(t + 1, mr);
          }
          const int cy = 2 * oy - 1 + ky;  // conv1 output row of this tap (wave-uniform)
#pragma unroll
          for (int mr = 0; mr < 4; ++mr) {
            const bf16x8 a1 = __builtin_bit_cast(bf16x8, pw[cur][mr]);
            const f32x4 d0 = mfma(bw1[0], a1, bv1[0]);
            const f32x4 d1 = mfma(bw1[1], a1, bv1[1]);
            uint4 pk;
            pk.x = relu_bf16x2(pack_bf16x2(d0[0], d0[1]));
            pk.y = relu_bf16x2(pack_bf16x2(d0[2], d0[3]));
            pk.z = relu_bf16x2(pack_bf16x2(d1[0], d1[1]));
            pk.w = relu_bf16x2(pack_bf16x2(d1[2], d1[3]));
            if constexpr (EDGE) {
              const int cx = xb + 1 + 2 * (mr * 16 + r16) + kx;  // conv1 output column
              if (cy < 0 || cy >= g1.ho || cx < 0 || cx >= g1.wo) pk = make_uint4(0u, 0u, 0u, 0u);
            }
            const bf16x8 a2 = __builtin_bit_cast(bf16x8, pk);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[mr][nb] = mfma(bq[nb], a2, acc[mr][nb]);
          }
          // keep each tap's fragment reads with its MFMAs (hoisting every tap's
          // reads ahead would hold 9 x 16 fragment registers)
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (col_edge || oy == 0) taps(std::true_type{});
      else taps(std::false_type{});
      char* yimg = reinterpret_cast<char*>(y) + (int64_t)n * g2.ho * g2.wo * 64 * 2;  // wave-uniform
#pragma unroll
      for (int mr = 0; mr < 4; ++mr) {
        const int ox = ox0 + mr * 16 + r16;
        if (ox >= g2.wo || mr * 16 + r16 >= kC12sStep) continue;
        const uint32_t mo = (uint32_t)(oy * g2.wo + ox) * (uint32_t)(64 * 2);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const f32x4 v = acc[mr][nb];  // bias included
          typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
          stg32(reinterpret_cast<u32x2_t*>(yimg), mo + 2u * (uint32_t)(nb * 16 + 4 * kg),
                u32x2_t{relu_bf16x2(pack_bf16x2(v[0], v[1])), relu_bf16x2(pack_bf16x2(v[2], v[3]))});
        }
      }
      // rows 2oy+3, 2oy+4 take the slots of rows 2oy-5, 2oy-4, which no
      // tap of this output row read (a wave's LDS operations run in order)
      store_row(2 * oy + 3, nx[0]);
      store_row(2 * oy + 4, nx[1]);
    }
  }
}

// ---------------------------------------------------------------------------
// input gradient of the effective input: dxe[m][ci] = sum_{tap, co} W[tap][co][ci] dy(out(m, tap))[co]
template <int L, int MR, bool FUSE>
__global__ void __launch_bounds__(256) k_conv_dx(const void* __restrict__ dy, const uint8_t* __restrict__ blob,
                                                 float* __restrict__ dxe, CGeom g, const bf16_t* __restrict__ act,
                                                 bf16_t* __restrict__ gout) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, NB = CI / 16;
  static_assert(CI % 16 == 0, "input-gradient kernel needs ci % 16 == 0");
  // FUSE (layers that read their input without upsampling): the previous
  // layer's output gradient is formed here -- times the ReLU derivative of
  // its stored activation `act`, rounded to BF16 into `gout` -- instead of
  // going through dxe and k_dx_post (the same values)
  static_assert(!FUSE || !D.up, "the upsampling adjoint needs k_dx_post");
  const bf16_t* wt = reinterpret_cast<const bf16_t*>(blob + blob_tr_off(L));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t M = (int64_t)g.n * g.he * g.we;
  const int64_t base = ((int64_t)blockIdx.x * 4 + wv) * (16 * MR);
  int pn[MR], piy[MR], pix[MR];
  bool pv[MR];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr) {
    const int64_t m = base + mr * 16 + r16;
    pv[mr] = m < M;
    const int64_t mm = pv[mr] ? m : 0;
    pix[mr] = (int)(mm % g.we);
    const int64_t t = mm / g.we;
    piy[mr] = (int)(t % g.he);
    pn[mr] = (int)(t / g.he);
  }
  f32x4 acc[MR][NB];
#pragma unroll
  for (int mr = 0; mr < MR; ++mr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mr][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto out_of = [&](int iv, int k, int n_out, int* o) -> bool {
    const int num = iv + 1 - k;
    if (num < 0) return false;
    if (S == 2) {
      if (num & 1) return false;
      *o = num >> 1;
    } else {
      *o = num;
    }
    return *o < n_out;
  };
  if constexpr (CO == 2) {
    // K = 18 (9 taps x 2 output channels) in one block of 32; dy is FP32 [m][2].
    const float* dyf = reinterpret_cast<const float*>(dy);
    bf16x8 a[MR];
#pragma unroll
    for (int mr = 0; mr < MR; ++mr) {
      bf16_t v[8];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int tap = 4 * kg + j;
        float d0 = 0.f, d1 = 0.f;
        int oy, ox;
        if (tap < 9 && pv[mr] && out_of(piy[mr], tap / 3, g.ho, &oy) && out_of(pix[mr], tap % 3, g.wo, &ox)) {
          const float2 d = *reinterpret_cast<const float2*>(dyf + (((int64_t)pn[mr] * g.ho + oy) * g.wo + ox) * 2);
          d0 = d.x;
          d1 = d.y;
        }
        v[2 * j] = f2bf(d0);
        v[2 * j + 1] = f2bf(d1);
      }
      a[mr] = pack8(v);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 b = ld8(wt + (nb * 16 + r16) * 32 + kg * 8);
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) acc[mr][nb] = mfma(a[mr], b, acc[mr][nb]);
    }
  } else {
    const bf16_t* dyb = reinterpret_cast<const bf16_t*>(dy);
    for (int tap = 0; tap < 9; ++tap) {
      int64_t off[MR];
      bool ok[MR];
#pragma unroll
      for (int mr = 0; mr < MR; ++mr) {
        int oy = 0, ox = 0;
        ok[mr] = pv[mr] && out_of(piy[mr], tap / 3, g.ho, &oy) && out_of(pix[mr], tap % 3, g.wo, &ox);
        off[mr] = ok[mr] ? (((int64_t)pn[mr] * g.ho + oy) * g.wo + ox) * CO : 0;
      }
#pragma unroll
      for (int cb = 0; cb < CO / 32; ++cb) {
        bf16x8 a[MR];
#pragma unroll
        for (int mr = 0; mr < MR; ++mr) a[mr] = ok[mr] ? ld8(dyb + off[mr] + cb * 32 + kg * 8) : zero8();
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bf16x8 b = ld8(wt + ((int64_t)(tap * CI + nb * 16 + r16) * CO + cb * 32 + kg * 8));
#pragma unroll
          for (int mr = 0; mr < MR; ++mr) acc[mr][nb] = mfma(a[mr], b, acc[mr][nb]);
        }
      }
    }
  }
#pragma unroll
  for (int mr = 0; mr < MR; ++mr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = base + mr * 16 + kg * 4 + i;
        if (m >= M) continue;
        const int64_t o = m * CI + nb * 16 + r16;
        if constexpr (FUSE) gout[o] = bf2f(act[o]) > 0.f ? f2bf(acc[mr][nb][i]) : (bf16_t)0;
        else dxe[o] = acc[mr][nb][i];
      }
}

// previous layer's output gradient: adjoint of the x2 upsampling (if any),
// times the ReLU derivative of the stored activation, rounded to BF16.
// One thread per 8 consecutive channels of one pixel (channel counts are
// multiples of 8): two 16-byte loads per FP32 row of 8 (four rows under the
// upsampling adjoint), one 16-byte load of the activation, one 16-byte store.
__global__ void k_dx_post(const float* __restrict__ dxe, const bf16_t* __restrict__ act, bf16_t* __restrict__ gout,
                          int64_t n_groups, int32_t h, int32_t w, int32_t c, int32_t up) {
  const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gi >= n_groups) return;
  const int32_t g8 = c >> 3;
  const int64_t p = gi / g8;  // pixel (n, y, x) at the gradient's resolution
  const int32_t ch = (int32_t)(gi - p * g8) << 3;
  typedef float f32x4_t __attribute__((ext_vector_type(4)));
  auto row8 = [&](int64_t off, float (&r)[8]) {
    const f32x4_t lo = *reinterpret_cast<const f32x4_t*>(dxe + off);
    const f32x4_t hi = *reinterpret_cast<const f32x4_t*>(dxe + off + 4);
    r[0] = lo.x; r[1] = lo.y; r[2] = lo.z; r[3] = lo.w;
    r[4] = hi.x; r[5] = hi.y; r[6] = hi.z; r[7] = hi.w;
  };
  float v[8];
  if (up) {
    const int64_t t = p / w, n = t / h;
    const int32_t xx = (int32_t)(p - t * w), yy = (int32_t)(t - n * h);
    const int64_t W2 = 2 * (int64_t)w, H2 = 2 * (int64_t)h;
    const int64_t b = ((n * H2 + 2 * yy) * W2 + 2 * xx) * c + ch;
    float r00[8], r01[8], r10[8], r11[8];
    row8(b, r00);
    row8(b + c, r01);
    row8(b + W2 * c, r10);
    row8(b + W2 * c + c, r11);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (r00[k] + r01[k]) + (r10[k] + r11[k]);
  } else {
    row8(p * c + ch, v);
  }
  const uint4 a = *reinterpret_cast<const uint4*>(act + p * c + ch);
  const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bf16_t lo = bf2f((bf16_t)(aw[k] & 0xFFFFu)) > 0.f ? f2bf(v[2 * k]) : (bf16_t)0;
    const bf16_t hi = bf2f((bf16_t)(aw[k] >> 16)) > 0.f ? f2bf(v[2 * k + 1]) : (bf16_t)0;
    o[k] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
  *reinterpret_cast<uint4*>(gout + p * c + ch) = make_uint4(o[0], o[1], o[2], o[3]);
}

// ---------------------------------------------------------------------------
// weight gradient, split over chunks of whole output rows (deterministic):
//   part[chunk][tap][co][ci] = sum_{m in chunk} dy[m][co] x_e(m, tap)[ci]
//   partb[chunk][co] = sum_{m in chunk} dy[m][co]
// A workgroup computes the taps of TR tap rows of one chunk (all nine, or
// one tap row for the two layers with 64 x 96 channel pairs, whose
// accumulators would not fit otherwise).  It walks steps of 32
// output pixels of one row; per step dy and the nine taps' inputs are staged
// transposed to [channel][pixel] in LDS (8 consecutive pixels of a channel
// are one 16-byte MFMA fragment, K = pixels): 16-byte loads of 8 channels of
// 8 pixels are transposed in registers with byte permutes and stored as 8
// 16-byte rows.  The next step's loads are in flight during this step's
// MFMAs.  conv1's 2-channel input and conv6's FP32 2-channel dy are staged
// element-wise (their other channel rows stay zero).
constexpr int64_t kDwMaxChunks = 512;  // weight-gradient workgroups per layer (at most)
inline int64_t dw_rows_per_chunk(int64_t rows) { return std::max<int64_t>(1, (rows + kDwMaxChunks - 1) / kDwMaxChunks); }
inline int64_t dw_chunks(int64_t rows) { return (rows + dw_rows_per_chunk(rows) - 1) / dw_rows_per_chunk(rows); }

// 8 x 8 transpose of 16-bit elements: in[j] holds channels 0..7 of pixel j,
// out[c] receives pixels 0..7 of channel c.
__device__ __forceinline__ void transpose8x8(const uint4 (&in)[8], uint4 (&out)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;  // high or low halves of the two dwords
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 a = in[2 * k], b = in[2 * k + 1];
      const uint32_t da = (c >> 1) == 0 ? a.x : (c >> 1) == 1 ? a.y : (c >> 1) == 2 ? a.z : a.w;
      const uint32_t db = (c >> 1) == 0 ? b.x : (c >> 1) == 1 ? b.y : (c >> 1) == 2 ? b.z : b.w;
      w[k] = __builtin_amdgcn_perm(db, da, sel);  // low 16 bits from pixel 2k, high 16 bits from pixel 2k + 1
    }
    out[c] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int L, int NW, int TR>
__global__ void __launch_bounds__(64 * NW) k_conv_dw(const void* __restrict__ dy, const bf16_t* __restrict__ x,
                                                     float* __restrict__ part, float* __restrict__ partb, CGeom g,
                                                     int32_t rows_per_chunk) {
  constexpr LayerDef D = kNet[L];
  constexpr int CI = D.ci, CO = D.co, S = D.stride, COP = cpad(CO), CIP = cpad(CI);
  constexpr bool UP = D.up != 0;
  constexpr bool DY32 = L == kLayers - 1;  // conv6: dy is the FP32 gradient of the 2-channel flow
  constexpr bool XS = CI < 8;              // conv1: 2 input channels
  static_assert(DY32 ? CO == 2 : CO % 8 == 0, "dy staging");
  static_assert(XS ? CI == 2 : CI % 8 == 0, "input staging");
  constexpr int NT = 64 * NW, LS = 40;  // staged rows: 32 pixels + padding (80-byte rows)
  constexpr int NTAP = 3 * TR;  // taps of this workgroup: tap rows ky0 .. ky0 + TR - 1
  constexpr int TCO = COP / 16, TCI = CIP / 16, NTILE = NTAP * TCO * TCI, TPW = (NTILE + NW - 1) / NW;
  // staging units of a step: dy (8 x 8 blocks, or one pixel for DY32) then x
  // (tap x 8 x 8 blocks, or tap x one pixel for XS)
  constexpr int NDY = DY32 ? 32 : 4 * (CO / 8);
  constexpr int NXU = XS ? NTAP * 32 : NTAP * 4 * (CI / 8);
  constexpr int NU = NDY + NXU, UPT = (NU + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) bf16_t sdy[COP][LS];
  __shared__ __attribute__((aligned(16))) bf16_t sx[NTAP][CIP][LS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t rows = (int64_t)g.n * g.ho;
  const int64_t chunk = blockIdx.x / (3 / TR);
  const int ky0 = (int)(blockIdx.x % (3 / TR)) * TR;
  const int64_t r0 = chunk * rows_per_chunk, r1 = min(rows, r0 + rows_per_chunk);
  const int nxb = (g.wo + 31) / 32;
  const int nsteps = (int)(r1 - r0) * nxb;
  // channel rows no unit writes (padding of 2-channel operands) stay zero
  if constexpr (DY32)
    for (int e = tid; e < (COP - CO) * LS; e += NT) sdy[CO + e / LS][e % LS] = 0;
  if constexpr (XS)
    for (int e = tid; e < NTAP * (CIP - CI) * LS; e += NT) {
      const int t = e / ((CIP - CI) * LS), rem = e % ((CIP - CI) * LS);
      sx[t][CI + rem / LS][rem % LS] = 0;
    }

  uint4 ureg[UPT][8];  // loaded units (element-wise units use the first words)
  auto load = [&](int st) {
    const int64_t r = r0 + st / nxb;
    const int xb = st % nxb;
    const int n = (int)(r / g.ho), oy = (int)(r % g.ho);
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * NT;
      if (u >= NU) continue;
      if (u < NDY) {
        if constexpr (DY32) {
          const int ox = xb * 32 + u;
          float2 v = make_float2(0.f, 0.f);
          if (ox < g.wo)
            v = reinterpret_cast<const float2*>(dy)[((int64_t)n * g.ho + oy) * g.wo + ox];
          ureg[k][0] = make_uint4(f2bf(v.x), f2bf(v.y), 0, 0);
        } else {
          const int pg = u / (CO / 8), cg = u % (CO / 8);
          const bf16_t* base = reinterpret_cast<const bf16_t*>(dy) + (((int64_t)n * g.ho + oy) * g.wo) * CO + 8 * cg;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int ox = xb * 32 + 8 * pg + j;
            ureg[k][j] = ox < g.wo ? *reinterpret_cast<const uint4*>(base + (int64_t)ox * CO) : make_uint4(0, 0, 0, 0);
          }
        }
      } else {
        const int v = u - NDY;
        if constexpr (XS) {
          const int tap = v / 32, p = v % 32, ky = ky0 + tap / 3, kx = tap % 3;
          const int ox = xb * 32 + p;
          const int iy = oy * S + ky - 1, ix = ox * S + kx - 1;
          uint32_t w = 0;
          if (ox < g.wo && iy >= 0 && iy < g.he && ix >= 0 && ix < g.we) {
            const int sy = UP ? iy >> 1 : iy, sxx = UP ? ix >> 1 : ix;
            w = *reinterpret_cast<const uint32_t*>(x + (((int64_t)n * g.hi + sy) * g.wi + sxx) * CI);
          }
          ureg[k][0] = make_uint4(w, 0, 0, 0);
        } else {
          const int tap = v / (4 * (CI / 8)), rem = v % (4 * (CI / 8));
          const int pg = rem / (CI / 8), cg = rem % (CI / 8), ky = ky0 + tap / 3, kx = tap % 3;
          const int iy = oy * S + ky - 1;
          const bool row_in = iy >= 0 && iy < g.he;
          const int sy = UP ? iy >> 1 : iy;
          const bf16_t* base = x + ((int64_t)n * g.hi + (row_in ? sy : 0)) * g.wi * CI + 8 * cg;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int ox = xb * 32 + 8 * pg + j, ix = ox * S + kx - 1;
            const bool ok = row_in && ox < g.wo && ix >= 0 && ix < g.we;
            const int sxx = UP ? ix >> 1 : ix;
            ureg[k][j] = ok ? *reinterpret_cast<const uint4*>(base + (int64_t)sxx * CI) : make_uint4(0, 0, 0, 0);
          }
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * NT;
      if (u >= NU) continue;
      if (u < NDY) {
        if constexpr (DY32) {
          sdy[0][u] = (bf16_t)ureg[k][0].x;
          sdy[1][u] = (bf16_t)ureg[k][0].y;
        } else {
          const int pg = u / (CO / 8), cg = u % (CO / 8);
          uint4 t8[8];
          transpose8x8(ureg[k], t8);
#pragma unroll
          for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4*>(&sdy[8 * cg + c][8 * pg]) = t8[c];
        }
      } else {
        const int v = u - NDY;
        if constexpr (XS) {
          const int tap = v / 32, p = v % 32;
          sx[tap][0][p] = (bf16_t)(ureg[k][0].x & 0xFFFFu);
          sx[tap][1][p] = (bf16_t)(ureg[k][0].x >> 16);
        } else {
          const int tap = v / (4 * (CI / 8)), rem = v % (4 * (CI / 8));
          const int pg = rem / (CI / 8), cg = rem % (CI / 8);
          uint4 t8[8];
          transpose8x8(ureg[k], t8);
#pragma unroll
          for (int c = 0; c < 8; ++c) *reinterpret_cast<uint4*>(&sx[tap][8 * cg + c][8 * pg]) = t8[c];
        }
      }
    }
  };

  f32x4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  if (nsteps > 0) load(0);
  for (int st = 0; st < nsteps; ++st) {
    store();
    __syncthreads();
    if (st + 1 < nsteps) load(st + 1);  // in flight during this step's MFMAs
    if (tid < CO) {
#pragma unroll 8
      for (int p = 0; p < 32; ++p) bsum += bf2f(sdy[tid][p]);
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = wv + NW * t;
      if (tile < NTILE) {
        const int tap = tile / (TCO * TCI), rem = tile % (TCO * TCI);
        const int tco = rem / TCI, tci = rem % TCI;
        const bf16x8 a = ld8(&sdy[tco * 16 + r16][kg * 8]);
        const bf16x8 b = ld8(&sx[tap][tci * 16 + r16][kg * 8]);
        acc[t] = mfma(a, b, acc[t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wv + NW * t;
    if (tile >= NTILE) continue;
    const int tap = 3 * ky0 + tile / (TCO * TCI), rem = tile % (TCO * TCI);
    const int tco = rem / TCI, tci = rem % TCI;
    const int ci = tci * 16 + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = tco * 16 + kg * 4 + i;
      if (co < CO && ci < CI) part[((chunk * 9 + tap) * CO + co) * CI + ci] = acc[t][i];
    }
  }
  if (ky0 == 0 && tid < CO) partb[chunk * CO + tid] = bsum;
}

// Chunk partials are summed in two deterministic stages: groups of
// kDwGroup consecutive chunks (in place: group g's sum replaces the partial
// of its first chunk, which only that group reads), then the group sums in
// group order.  One thread per weight or bias element per stage.
constexpr int64_t kDwGroup = 32;
__global__ void k_dw_group(float* __restrict__ part, float* __restrict__ partb, int64_t chunks, int64_t nw,
                           int32_t co) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * kDwGroup, k1 = min(chunks, k0 + kDwGroup);
  if (i < nw) {
    float s = 0.f;
    for (int64_t k = k0; k < k1; ++k) s += part[k * nw + i];
    part[k0 * nw + i] = s;
  } else if (i < nw + co) {
    const int64_t c = i - nw;
    float s = 0.f;
    for (int64_t k = k0; k < k1; ++k) s += partb[k * co + c];
    partb[k0 * co + c] = s;
  }
}

// Group sums, in group order, into the gradient vector (master layout
// [co][ci][ky][kx]).  Thread i takes partial index i ([tap][co][ci] order),
// so that a wave reads consecutive floats of every group.
__global__ void k_dw_reduce(const float* __restrict__ part, const float* __restrict__ partb, float* __restrict__ grads,
                            int64_t chunks, int32_t ci, int32_t co, int32_t w_off, int32_t b_off) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)co * ci * 9;
  if (i < nw) {
    const int c_in = (int)(i % ci);
    const int64_t t = i / ci;
    const int c_out = (int)(t % co), tap = (int)(t / co);
    float s = 0.f;
    for (int64_t k = 0; k < chunks; k += kDwGroup) s += part[k * nw + i];
    grads[w_off + ((int64_t)c_out * ci + c_in) * 9 + tap] = s;
  } else if (i < nw + co) {
    const int c_out = (int)(i - nw);
    float s = 0.f;
    for (int64_t k = 0; k < chunks; k += kDwGroup) s += partb[k * co + c_out];
    grads[b_off + c_out] = s;
  }
}

// ---------------------------------------------------------------------------
// network input: per pair, 2x2 mean of each frame's luma (round half up) as (v - 128)/64 in BF16.
__global__ void k_net_input(const FrameDesc* __restrict__ frames, const PairDesc* __restrict__ pairs,
                            bf16_t* __restrict__ x, int32_t h, int32_t w, int64_t n_pairs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_pairs * h * w) return;
  const int32_t xx = (int32_t)(i % w);
  const int64_t t = i / w;
  const int32_t yy = (int32_t)(t % h);
  const int64_t p = t / h;
  bf16_t out[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const FrameDesc fd = frames[f == 0 ? pairs[p].f1 : pairs[p].f2];
    const uint8_t* r0 = fd.y + (int64_t)(2 * yy) * fd.pitch + 2 * xx;
    const int s = (int)r0[0] + r0[1] + r0[fd.pitch] + r0[fd.pitch + 1];
    out[f] = f2bf((float)(((s + 2) >> 2) - 128) * (1.f / 64.f));
  }
  *reinterpret_cast<uint32_t*>(x + i * 2) = (uint32_t)out[0] | ((uint32_t)out[1] << 16);
}

// pixels per thread of the fused upsample + gate kernel (4 ran no faster:
// more waves per SIMD, but 16% more VALU work per pixel)
constexpr int kGateGX = 2, kGateGY = 1, kGatePx = 4 * kGateGX * kGateGY;

// Bilinear x2 upsampling tap (half-pixel centres, clamped).
struct UpTap {
  int i0, i1;
  float f;
};
__device__ __forceinline__ UpTap up_tap(int x, int n_half) {
  float X = ((float)x + 0.5f) * 0.5f - 0.5f;
  X = fminf(fmaxf(X, 0.f), (float)(n_half - 1));
  UpTap t;
  t.i0 = (int)floorf(X);
  t.i1 = min(t.i0 + 1, n_half - 1);
  t.f = X - (float)t.i0;
  return t;
}

__device__ __forceinline__ float2 full_flow_at(const float* __restrict__ half, int x, int y, int h, int w) {
  const UpTap tx = up_tap(x, w), ty = up_tap(y, h);
  const float2 a = *reinterpret_cast<const float2*>(half + ((int64_t)ty.i0 * w + tx.i0) * 2);
  const float2 b = *reinterpret_cast<const float2*>(half + ((int64_t)ty.i0 * w + tx.i1) * 2);
  const float2 c = *reinterpret_cast<const float2*>(half + ((int64_t)ty.i1 * w + tx.i0) * 2);
  const float2 d = *reinterpret_cast<const float2*>(half + ((int64_t)ty.i1 * w + tx.i1) * 2);
  const float u = (1.f - ty.f) * ((1.f - tx.f) * a.x + tx.f * b.x) + ty.f * ((1.f - tx.f) * c.x + tx.f * d.x);
  const float v = (1.f - ty.f) * ((1.f - tx.f) * a.y + tx.f * b.y) + ty.f * ((1.f - tx.f) * c.y + tx.f * d.y);
  return make_float2(2.f * u, 2.f * v);
}

// full-resolution flow [2][H][W] per pair from the half-resolution output [h][w][2];
// pairs whose keep flag is 0 are skipped (their output comes from elsewhere).
__global__ void k_flow_up(const float* __restrict__ half, const PairDesc* __restrict__ pairs, int32_t h, int32_t w,
                          int64_t n_pairs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int32_t W = 2 * w, H = 2 * h;
  if (i >= n_pairs * H * W) return;
  const int32_t x = (int32_t)(i % W);
  const int64_t t = i / W;
  const int32_t y = (int32_t)(t % H);
  const int64_t p = t / H;
  const float2 f = full_flow_at(half + p * (int64_t)h * w * 2, x, y, h, w);
  float* out = pairs[p].out;
  out[(int64_t)y * W + x] = f.x;
  out[(int64_t)H * W + (int64_t)y * W + x] = f.y;
}

// Charbonnier loss against the target flow and its gradient w.r.t. the
// half-resolution output (adjoint of the x2 upsampling, gathered per half
// pixel).  Full pixel (x, y) counts its loss term at half pixel (x/2, y/2).
__global__ void k_loss_grad(const float* __restrict__ half, const PairDesc* __restrict__ pairs,
                            float* __restrict__ ghalf, float* __restrict__ loss_part, int32_t h, int32_t w,
                            int64_t n_pairs, float scale) {
  __shared__ float red[256];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float own = 0.f;
  if (i < n_pairs * h * w) {
    const int32_t hx = (int32_t)(i % w);
    const int64_t t = i / w;
    const int32_t hy = (int32_t)(t % h);
    const int64_t p = t / h;
    const int32_t W = 2 * w, H = 2 * h;
    const float* hp = half + p * (int64_t)h * w * 2;
    const float* tg = pairs[p].out;
    float gu = 0.f, gv = 0.f;
    for (int y = max(2 * hy - 2, 0); y <= min(2 * hy + 2, H - 1); ++y) {
      const UpTap ty = up_tap(y, h);
      const float wy = (ty.i0 == hy ? 1.f - ty.f : 0.f) + (ty.i1 == hy ? ty.f : 0.f);
      for (int x = max(2 * hx - 2, 0); x <= min(2 * hx + 2, W - 1); ++x) {
        const UpTap tx = up_tap(x, w);
        const float wx = (tx.i0 == hx ? 1.f - tx.f : 0.f) + (tx.i1 == hx ? tx.f : 0.f);
        const bool owned = (x >> 1) == hx && (y >> 1) == hy;
        if (wx * wy == 0.f && !owned) continue;
        const float2 f = full_flow_at(hp, x, y, h, w);
        const float du = f.x - tg[(int64_t)y * W + x];
        const float dv = f.y - tg[(int64_t)H * W + (int64_t)y * W + x];
        const float r = sqrtf(du * du + dv * dv + 1e-4f);
        if (owned) own += r;
        const float k = 2.f * wx * wy * scale / r;
        gu += k * du;
        gv += k * dv;
      }
    }
    ghalf[i * 2] = gu;
    ghalf[i * 2 + 1] = gv;
  }
  red[threadIdx.x] = own;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_sum_loss(const float* __restrict__ part, int64_t n, float scale, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

// ---------------------------------------------------------------------------
// pack FP32 master weights into the BF16 blob (forward and transposed layouts) + FP32 bias
__device__ void pack_one(int64_t i, float wv, uint8_t* blob) {
  for (int l = 0; l < kLayers; ++l) {
    const int ci = kNet[l].ci, co = kNet[l].co;
    const int64_t wo = param_w_off(l), bo = param_b_off(l);
    if (i >= wo && i < bo) {
      const int64_t j = i - wo;
      const int tap = (int)(j % 9);
      const int64_t t = j / 9;
      const int c_in = (int)(t % ci), c_out = (int)(t / ci);
      const bf16_t b = f2bf(wv);
      bf16_t* wf = reinterpret_cast<bf16_t*>(blob + blob_fwd_off(l));
      bf16_t* wt = reinterpret_cast<bf16_t*>(blob + blob_tr_off(l));
      if (ci == 2)
        wf[c_out * 32 + 2 * tap + c_in] = b;
      else
        wf[((int64_t)tap * cpad(co) + c_out) * ci + c_in] = b;
      if (co == 2)
        wt[c_in * 32 + 2 * tap + c_out] = b;
      else
        wt[((int64_t)tap * ci + c_in) * co + c_out] = b;
      return;
    }
    if (i >= bo && i < bo + co) {
      reinterpret_cast<float*>(blob + blob_bias_off(l))[i - bo] = wv;
      return;
    }
  }
}

__global__ void k_pack(const float* __restrict__ master, uint8_t* __restrict__ blob) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < kParams) pack_one(i, master[i], blob);
}

__global__ void k_zero_bytes(uint32_t* __restrict__ p, int64_t n_words) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n_words) p[i] = 0u;
}

__global__ void k_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float bc1, float bc2,
                       uint8_t* __restrict__ blob) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  master[i] = w;
  pack_one(i, w, blob);
}

// ---------------------------------------------------------------------------
// residual gate: per pair, mean |I2(x + w) - I1(x)| over full-resolution luma
// (clamped bilinear warp), in two deterministic stages.
// Full-resolution flow of the network (x2 bilinear of the half-resolution
// output, written to the pair's output) fused with the gate statistic
// |I2(x + w) - I1(x)| (clamped bilinear warp of luma), reduced per block.
template <int GX, int GY>
__global__ void __launch_bounds__(256) k_up_gate(const float* __restrict__ half, const FrameDesc* __restrict__ frames,
                                                 const PairDesc* __restrict__ pairs, float* __restrict__ part,
                                                 int32_t h, int32_t w, int32_t blocks_per_pair) {
  // Each thread: GX x GY groups of 4 consecutive pixels, the groups W / GX
  // columns and H / GY rows apart (W is a multiple of 4 GX, H of GY), so that
  // the 16-byte flow stores of consecutive threads cover consecutive memory
  // and each thread has GX GY independent groups of loads in flight.
  static_assert(GX >= 1 && GX <= 2 && GY >= 1 && GY <= 2, "groups per thread");
  __shared__ float red[4];
  const int32_t W = 2 * w, H = 2 * h;
  const int32_t TPR = W / (4 * GX), RPG = H / GY;  // threads per row, rows per row group
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t p = blk / blocks_per_pair;
  const int32_t q = (blk % blocks_per_pair) * 256 + threadIdx.x;
  float r = 0.f;
  if (q < TPR * RPG) {
    const int32_t yq = q / TPR, t = q % TPR;
    const PairDesc pd = pairs[p];
    const FrameDesc f1 = frames[pd.f1], f2 = frames[pd.f2];
    const float* hp = half + p * (int64_t)h * w * 2;
    const uint8_t* a = f2.y;
    const uint32_t p2 = (uint32_t)f2.pitch;
    const bool al4 = ((reinterpret_cast<uintptr_t>(f1.y) | (uintptr_t)f1.pitch) & 3) == 0;
#pragma unroll
    for (int gi = 0; gi < GX * GY; ++gi) {
      const int32_t xb = 4 * t + (gi % GX) * (W / GX), y = yq + (gi / GX) * RPG;
      const uint8_t* row1 = f1.y + y * (int32_t)f1.pitch;
      const UpTap ty = up_tap(y, h);
      const uint32_t o_u = 4u * (uint32_t)(y * W), o_v = o_u + 4u * (uint32_t)(W * H);  // byte offsets of the row
      // the first frame's 4 luma bytes in one load where the row is aligned
      uint8_t y1v[4];
      if (al4) {
        const uint32_t v4 = ldg32(reinterpret_cast<const uint32_t*>(row1), (uint32_t)xb);
#pragma unroll
        for (int k = 0; k < 4; ++k) y1v[k] = (uint8_t)(v4 >> (8 * k));
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) y1v[k] = ldg32(row1, (uint32_t)(xb + k));
      }
      // The 4 pixels read half-resolution columns k0 .. k0 + 3 (k0 = xb/2 - 1,
      // clamped) of two rows: 8 loads instead of 16.  Pixel j's taps (up_tap)
      // are columns (j+1)/2 and (j+1)/2 + 1 of that window; at the clamped
      // image borders the tap weight of a substituted column is 0, so the
      // values equal full_flow_at's.
      const int32_t k0 = xb / 2 - 1;
      float2 r0[4], r1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int32_t col = min(max(k0 + c, 0), w - 1);
        const f32x2_t t0 = ldg32(reinterpret_cast<const f32x2_t*>(hp), 8u * ((uint32_t)ty.i0 * (uint32_t)w + (uint32_t)col));
        const f32x2_t t1 = ldg32(reinterpret_cast<const f32x2_t*>(hp), 8u * ((uint32_t)ty.i1 * (uint32_t)w + (uint32_t)col));
        r0[c] = make_float2(t0.x, t0.y);
        r1[c] = make_float2(t1.x, t1.y);
      }
      // Away from the left and right image borders the horizontal taps are
      // fixed: weights 0.75 / 0.25 for even / odd pixels (exact values of
      // up_tap there), so the per-pixel tap arithmetic is skipped.
      const bool interior = xb > 0 && xb + 4 < W;
      float fu4[4], fv4[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t x = xb + k;
        UpTap tx;
        if (interior) tx.f = (k & 1) ? 0.25f : 0.75f;
        else tx = up_tap(x, w);
        constexpr int kIa[4] = {0, 1, 1, 2};
        const float2 fa = r0[kIa[k]], fb = r0[kIa[k] + 1], fc = r1[kIa[k]], fd = r1[kIa[k] + 1];
        const float uu = (1.f - ty.f) * ((1.f - tx.f) * fa.x + tx.f * fb.x) + ty.f * ((1.f - tx.f) * fc.x + tx.f * fd.x);
        const float vv = (1.f - ty.f) * ((1.f - tx.f) * fa.y + tx.f * fb.y) + ty.f * ((1.f - tx.f) * fc.y + tx.f * fd.y);
        const float2 f = make_float2(2.f * uu, 2.f * vv);
        fu4[k] = f.x;
        fv4[k] = f.y;
        const float fu = floorf(f.x), fv = floorf(f.y);
        int32_t xi = x + (int32_t)fu, yi = y + (int32_t)fv;
        float fx = f.x - fu, fy = f.y - fv;
        // Columns: the two samples of a row come from one 2-byte load at
        // xs = clamp(xi, 0, W - 2) (unaligned global loads are allowed).  Past
        // the right edge the clamped sample is the second byte with weight 1,
        // which equals the first byte with weight 0 of the plain clamped form.
        int32_t xs;
        if (xi < 0) { xs = 0; fx = 0.f; } else if (xi >= W - 1) { xs = W - 2; fx = 1.f; } else { xs = xi; }
        if (yi < 0) { yi = 0; fy = 0.f; } else if (yi >= H - 1) { yi = H - 1; fy = 0.f; }
        const int32_t y1 = min(yi + 1, H - 1);
        // rows < 2^15, pitch <= 2^20 (checked on the host): 24-bit products
        const uint32_t o0 = __umul24((uint32_t)yi, p2), o1 = __umul24((uint32_t)y1, p2);
        const uint32_t w0 = ldg32(reinterpret_cast<const uint16_t*>(a), o0 + (uint32_t)xs);
        const uint32_t w1 = ldg32(reinterpret_cast<const uint16_t*>(a), o1 + (uint32_t)xs);
        const float top = (1.f - fx) * (float)(w0 & 0xFFu) + fx * (float)(w0 >> 8);
        const float bot = (1.f - fx) * (float)(w1 & 0xFFu) + fx * (float)(w1 >> 8);
        r += fabsf((1.f - fy) * top + fy * bot - (float)y1v[k]);
      }
      typedef float f32x4_t __attribute__((ext_vector_type(4)));
      stg32(reinterpret_cast<f32x4_t*>(pd.out), o_u + 4u * (uint32_t)xb, f32x4_t{fu4[0], fu4[1], fu4[2], fu4[3]});
      stg32(reinterpret_cast<f32x4_t*>(pd.out), o_v + 4u * (uint32_t)xb, f32x4_t{fv4[0], fv4[1], fv4[2], fv4[3]});
    }
  }
  // wave reduction, then across the four waves (fixed order: deterministic)
  for (int off = 32; off > 0; off >>= 1) r += __shfl_down(r, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) part[blk] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One workgroup per pair: fixed-order strided sums, then a fixed tree, so the
// statistic is deterministic and the partials are read coalesced.
__global__ void __launch_bounds__(256) k_gate_final(const float* __restrict__ part, int32_t blocks_per_pair,
                                                    float inv_px, float tau, const PairDesc* __restrict__ pairs,
                                                    uint8_t* __restrict__ active) {
  __shared__ float red[4];
  const int64_t p = blockIdx.x;
  const float* src = part + p * blocks_per_pair;
  float s = 0.f;
  for (int b = threadIdx.x; b < blocks_per_pair; b += 256) s += src[b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const float r = ((red[0] + red[1]) + (red[2] + red[3])) * inv_px;
  const uint8_t a = r > tau ? 1 : 0;
  active[p] = a;
  const PairDesc pd = pairs[p];
  if (pd.resid) *pd.resid = r;
  if (pd.fb) *pd.fb = a;
}

// frame slots used by at least one active pair (factive zeroed beforehand)
__global__ void k_mark_frames(const PairDesc* __restrict__ pairs, const uint8_t* __restrict__ active,
                              uint8_t* __restrict__ factive, int64_t n_pairs) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n_pairs || !active[p]) return;
  factive[pairs[p].f1] = 1;
  factive[pairs[p].f2] = 1;
}

// The active pairs in ascending order and their count (one workgroup): each
// thread counts a contiguous run of flags, an exclusive scan of the 256
// counts gives each run's first list position, and the runs are written.
__global__ void __launch_bounds__(256) k_compact_active(const uint8_t* __restrict__ active, int64_t n_pairs,
                                                        int32_t* __restrict__ list, int32_t* __restrict__ count) {
  __shared__ int32_t part[256];
  const int t = threadIdx.x;
  const int64_t per = (n_pairs + 255) / 256, b0 = min(n_pairs, (int64_t)t * per), b1 = min(n_pairs, b0 + per);
  int32_t c = 0;
  for (int64_t i = b0; i < b1; ++i) c += active[i] != 0;
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan (Hillis-Steele)
    const int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t pos = part[t] - c;
  for (int64_t i = b0; i < b1; ++i)
    if (active[i]) list[pos++] = (int32_t)i;
  if (t == 255) *count = part[255];
}

}  // namespace

// ---------------------------------------------------------------------------
// host orchestration

struct NetBuffers {
  bf16_t* x;
  bf16_t* act[kLayers - 1];
  float* half;
  // training only
  float* ghalf;
  float* dxe;
  bf16_t* g[2];
  float* part;
  float* partb;
  float* loss_part;
};

struct NetDims {
  int32_t h, w;  // half resolution
  int32_t hl[kLayers + 1], wl[kLayers + 1];  // stored size of each layer's output (index l+1), input at 0
};

NetDims net_dims(int32_t W, int32_t H) {
  NetDims d;
  d.h = H / 2;
  d.w = W / 2;
  d.hl[0] = d.h;
  d.wl[0] = d.w;
  for (int l = 0; l < kLayers; ++l) {
    const int he = kNet[l].up ? 2 * d.hl[l] : d.hl[l], we = kNet[l].up ? 2 * d.wl[l] : d.wl[l];
    d.hl[l + 1] = (he - 1) / kNet[l].stride + 1;
    d.wl[l + 1] = (we - 1) / kNet[l].stride + 1;
  }
  return d;
}

struct NetLayout {
  size_t bytes = 0;
  size_t off_x = 0, off_act[kLayers - 1] = {}, off_half = 0, off_ghalf = 0, off_dxe = 0, off_g[2] = {}, off_part = 0,
         off_partb = 0, off_loss = 0;
};

NetLayout net_layout(int32_t W, int32_t H, int64_t n, bool training) {
  const NetDims d = net_dims(W, H);
  NetLayout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t r = o;
    o += align_up(b);
    return r;
  };
  L.off_x = take((size_t)n * d.h * d.w * 2 * 2);
  for (int l = 0; l < kLayers - 1; ++l) L.off_act[l] = take((size_t)n * d.hl[l + 1] * d.wl[l + 1] * kNet[l].co * 2);
  L.off_half = take((size_t)n * d.h * d.w * 2 * 4);
  if (training) {
    L.off_ghalf = take((size_t)n * d.h * d.w * 2 * 4);
    size_t dxe = 0, gmax = 0, part = 0, partb = 0;
    for (int l = 1; l < kLayers; ++l) {
      const int he = kNet[l].up ? 2 * d.hl[l] : d.hl[l], we = kNet[l].up ? 2 * d.wl[l] : d.wl[l];
      dxe = std::max(dxe, (size_t)n * he * we * kNet[l].ci * 4);
      gmax = std::max(gmax, (size_t)n * d.hl[l] * d.wl[l] * kNet[l].ci * 2);
    }
    for (int l = 0; l < kLayers; ++l) {
      const int64_t chunks = dw_chunks(n * (int64_t)d.hl[l + 1]);
      part = std::max(part, (size_t)chunks * 9 * kNet[l].co * kNet[l].ci * 4);
      partb = std::max(partb, (size_t)chunks * kNet[l].co * 4);
    }
    L.off_dxe = take(dxe);
    L.off_g[0] = take(gmax);
    L.off_g[1] = take(gmax);
    L.off_part = take(part);
    L.off_partb = take(partb);
    L.off_loss = take((size_t)((n * d.h * d.w + 255) / 256 + 1) * 4);
  }
  L.bytes = o;
  return L;
}

NetBuffers net_buffers(uint8_t* base, const NetLayout& L, bool training) {
  NetBuffers b{};
  b.x = reinterpret_cast<bf16_t*>(base + L.off_x);
  for (int l = 0; l < kLayers - 1; ++l) b.act[l] = reinterpret_cast<bf16_t*>(base + L.off_act[l]);
  b.half = reinterpret_cast<float*>(base + L.off_half);
  if (training) {
    b.ghalf = reinterpret_cast<float*>(base + L.off_ghalf);
    b.dxe = reinterpret_cast<float*>(base + L.off_dxe);
    b.g[0] = reinterpret_cast<bf16_t*>(base + L.off_g[0]);
    b.g[1] = reinterpret_cast<bf16_t*>(base + L.off_g[1]);
    b.part = reinterpret_cast<float*>(base + L.off_part);
    b.partb = reinterpret_cast<float*>(base + L.off_partb);
    b.loss_part = reinterpret_cast<float*>(base + L.off_loss);
  }
  return b;
}

CGeom layer_geom(const NetDims& d, int l, int64_t n) {
  CGeom g;
  g.n = (int32_t)n;
  g.hi = d.hl[l];
  g.wi = d.wl[l];
  g.he = kNet[l].up ? 2 * g.hi : g.hi;
  g.we = kNet[l].up ? 2 * g.wi : g.wi;
  g.ho = d.hl[l + 1];
  g.wo = d.wl[l + 1];
  return g;
}

constexpr int kMR = 4;  // 16-pixel row blocks per wave (conv1 forward in training, input gradients)

// Output tile (rows x columns), waves per workgroup and weights-in-LDS choice
// of the LDS-tiled forward kernel per layer (chosen by timing on the 1080p
// batch): conv4, conv5 and conv6 keep the whole weight tensor in LDS (conv4's
// 110 KB next to its quarter-size upsampled input tile); conv6 uses a 16 x 32
// output tile with 8 waves, conv4 8 x 32 with 8 waves (two pixel blocks per
// wave), conv5 8 x 32 with 4 waves (four blocks per wave, two workgroups per
// CU), the others 8 x 32 (4 x 32 for stride 2) with 4 waves; conv3 has a
// kernel of its own.  conv4 and conv5 run persistent (one workgroup per
// resident slot, weights staged once, next input tile loaded while the
// current one is multiplied); conv6, whose weights are small, is faster with
// one workgroup per tile.
template <int L> struct FwdTile {
  static constexpr bool BLDS = (L == 3 || L == 4 || L == 5);
  static constexpr bool PERS = (L == 3 || L == 4);
  // waves per SIMD the persistent kernel is compiled for (register budget
  // 512 / WPE): conv5 runs two 4-wave workgroups per CU (four pixel blocks
  // per wave, so each weight fragment read from LDS feeds more MFMAs), conv4
  // one 8-wave workgroup
  static constexpr int WPE = 2;
  static constexpr int TOH = kNet[L].stride == 2 ? 4 : (L == 5 ? 16 : 8), TOW = L == 2 ? 16 : 32;
  static constexpr int NWAVE = (L == 5 || L == 3) ? 8 : (L == 4 ? 4 : (L == 2 ? 2 : 4));
};

constexpr const char* kFwdTimer[kLayers] = {"conv_fwd1", "conv_fwd2", "conv_fwd3", "conv_fwd4", "conv_fwd5",
                                             "conv_fwd6"};

template <int L>
scn_status launch_fwd(const bf16_t* x, const uint8_t* blob, void* y, const CGeom& g, hipStream_t s) {
  KernelTimer timer("conv_fwd", s);
  KernelTimer timer_l(kFwdTimer[L], s);
  if constexpr (L == 0) {  // 2 input channels: K = 18 fits one MFMA K block, no tiling needed
    const int64_t M = (int64_t)g.n * g.ho * g.wo;
    const int64_t per_wg = 4 * 16 * kMR;
    const int64_t grid = (M + per_wg - 1) / per_wg;
    hipLaunchKernelGGL((k_conv_fwd<L, kMR>), dim3((unsigned)grid), dim3(256), 0, s, x, blob, y, g);
  } else {
    constexpr int TOH = FwdTile<L>::TOH, TOW = FwdTile<L>::TOW, NW = FwdTile<L>::NWAVE, WPE = FwdTile<L>::WPE;
    constexpr bool BL = FwdTile<L>::BLDS;
    const int32_t tx = (g.wo + TOW - 1) / TOW, ty = (g.ho + TOH - 1) / TOH;
    const int64_t grid = (int64_t)tx * ty * g.n;
    if (grid > 0x7FFFFFFF) { set_error("surrogate batch too large"); return SCN_EUNSUPPORTED; }
    if constexpr (L == 2) {
      // conv3: persistent, weights in LDS, one workgroup per CU
      constexpr int MR3 = 3;
      const int32_t tasks_x = (g.wo + 16 * MR3 - 1) / (16 * MR3);
      const int64_t n_tasks = (int64_t)g.n * g.ho * tasks_x;
      if (n_tasks > 0x7FFFFFFF) { set_error("surrogate batch too large"); return SCN_EUNSUPPORTED; }
      static std::map<int, int> resident3;
      static std::mutex mu3;
      int dev = 0, resident = 0;
      if (hipGetDevice(&dev) != hipSuccess) { set_error("HIP device query failed"); return SCN_EHIP; }
      {
        std::lock_guard<std::mutex> lk(mu3);
        resident = resident3[dev];
      }
      if (resident == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv_s2_pers<2, MR3>, 256, 0) != hipSuccess) {
          set_error("HIP device query failed");
          return SCN_EHIP;
        }
        resident = std::max(1, cus * std::max(1, per_cu));
        std::lock_guard<std::mutex> lk(mu3);
        resident3[dev] = resident;
      }
      const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>((n_tasks + 3) / 4, resident));
      hipLaunchKernelGGL((k_conv_s2_pers<2, MR3>), dim3((unsigned)wgs), dim3(256), 0, s, x, blob, (bf16_t*)y, g,
                         tasks_x, (int32_t)n_tasks);
    } else if constexpr (FwdTile<L>::PERS) {
      // persistent: as many workgroups as the device holds at once (queried
      // once per device)
      static std::map<int, int> resident_by_dev;
      static std::mutex mu;
      int resident = 0;
      {
        std::lock_guard<std::mutex> lk(mu);
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) { set_error("HIP device query failed"); return SCN_EHIP; }
        resident = resident_by_dev[dev];
      }
      if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv_fwd_pers<L, TOH, TOW, NW, WPE>, 64 * NW, 0) !=
                hipSuccess) {
          set_error("HIP device query failed");
          return SCN_EHIP;
        }
        resident = std::max(1, cus * std::max(1, per_cu));
        std::lock_guard<std::mutex> lk(mu);
        resident_by_dev[dev] = resident;
      }
      const int64_t wgs = std::min<int64_t>(grid, resident);
      hipLaunchKernelGGL((k_conv_fwd_pers<L, TOH, TOW, NW, WPE>), dim3((unsigned)wgs), dim3(64 * NW), 0, s, x, blob, y, g,
                         tx, tx * ty, (int32_t)grid);
    } else {
      hipLaunchKernelGGL((k_conv_fwd_lds<L, TOH, TOW, NW, BL>), dim3((unsigned)grid), dim3(64 * NW), 0, s, x, blob, y,
                         g, tx, tx * ty);
    }
  }
  SCN_LAUNCHED("conv forward launch");
  return SCN_OK;
}

template <int L>
scn_status launch_dx(const void* dy, const uint8_t* blob, float* dxe, const CGeom& g, hipStream_t s,
                     const bf16_t* act = nullptr, bf16_t* gout = nullptr) {
  const int64_t M = (int64_t)g.n * g.he * g.we;
  const int64_t per_wg = 4 * 16 * kMR;
  const int64_t grid = (M + per_wg - 1) / per_wg;
  KernelTimer timer("conv_dx", s);
  if (kNet[L].up && gout) {
    set_error("internal: an upsampling layer's input gradient needs the separate post-processing");
    return SCN_EINVAL;
  }
  if constexpr (!kNet[L].up) {
    if (gout) {
      hipLaunchKernelGGL((k_conv_dx<L, kMR, true>), dim3((unsigned)grid), dim3(256), 0, s, dy, blob, dxe, g, act,
                         gout);
      SCN_LAUNCHED("conv input-gradient launch");
      return SCN_OK;
    }
  }
  hipLaunchKernelGGL((k_conv_dx<L, kMR, false>), dim3((unsigned)grid), dim3(256), 0, s, dy, blob, dxe, g, act, gout);
  SCN_LAUNCHED("conv input-gradient launch");
  return SCN_OK;
}

template <int L>
scn_status launch_dw(const void* dy, const bf16_t* x, const NetBuffers& b, float* grads, const CGeom& g,
                     hipStream_t s) {
  const int64_t rows = (int64_t)g.n * g.ho;
  const int64_t rpc = dw_rows_per_chunk(rows), chunks = dw_chunks(rows);
  if (rows * g.wo > 0x7FFFFFFF) { set_error("surrogate batch too large"); return SCN_EUNSUPPORTED; }
  {
    // conv3 and conv4 (64 x 96 channel pairs): one tap row per workgroup
    constexpr int TR = (kNet[L].ci * kNet[L].co >= 64 * 96) ? 1 : 3;
    KernelTimer timer("conv_dw", s);
    hipLaunchKernelGGL((k_conv_dw<L, 4, TR>), dim3((unsigned)(chunks * (3 / TR))), dim3(256), 0, s, dy, x, b.part,
                       b.partb, g, (int32_t)rpc);
  }
  SCN_LAUNCHED("conv weight-gradient launch");
  const int64_t nw = (int64_t)kNet[L].co * kNet[L].ci * 9, n = nw + kNet[L].co;
  hipLaunchKernelGGL(k_dw_group, dim3((unsigned)((n + 255) / 256), (unsigned)((chunks + kDwGroup - 1) / kDwGroup)),
                     dim3(256), 0, s, b.part, b.partb, chunks, nw, kNet[L].co);
  SCN_LAUNCHED("weight-gradient group-sum launch");
  hipLaunchKernelGGL(k_dw_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b.part, b.partb, grads, chunks,
                     kNet[L].ci, kNet[L].co, param_w_off(L), param_b_off(L));
  SCN_LAUNCHED("weight-gradient reduce launch");
  return SCN_OK;
}

// Fused conv1 + conv2 (streaming): waves per workgroup, output rows per band,
// workgroups per CU (8-row bands balance the last round of waves better
// than 16- or 32-row ones; 4-row bands pay the five-row start too often).
constexpr int kC12sNW = 4, kC12sBand = 8, kC12sPerCu = 2;

scn_status launch_conv12(const FrameDesc* frames, const PairDesc* pairs, const uint8_t* blob, bf16_t* y,
                         const NetDims& d, int64_t n, hipStream_t s) {
  const CGeom g1 = layer_geom(d, 0, n), g2 = layer_geom(d, 1, n);
  const int32_t strips = (g2.wo + kC12sStep - 1) / kC12sStep, bands = (g2.ho + kC12sBand - 1) / kC12sBand;
  const int64_t units = (int64_t)strips * bands * n;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t grid = std::min<int64_t>((units + kC12sNW - 1) / kC12sNW, (int64_t)cus * kC12sPerCu);
  KernelTimer timer("conv_fwd", s);
  KernelTimer timer_l("conv_fwd12", s);
  hipLaunchKernelGGL((k_conv12s<kC12sNW, kC12sBand>), dim3((unsigned)grid), dim3(64 * kC12sNW), 0, s, frames, pairs,
                     blob, y, g1, g2, strips, bands, units);
  SCN_LAUNCHED("fused conv1 + conv2 launch");
  return SCN_OK;
}

// Inference forward: the network input, conv1 and conv2 in one kernel
// (neither the input nor conv1's activation is kept).
scn_status net_forward_infer(const FrameDesc* frames, const PairDesc* pairs, const NetDims& d, int64_t n,
                             const uint8_t* blob, const NetBuffers& b, hipStream_t s) {
  scn_status st;
  if ((st = launch_conv12(frames, pairs, blob, b.act[1], d, n, s)) != SCN_OK) return st;
  if ((st = launch_fwd<2>(b.act[1], blob, b.act[2], layer_geom(d, 2, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<3>(b.act[2], blob, b.act[3], layer_geom(d, 3, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<4>(b.act[3], blob, b.act[4], layer_geom(d, 4, n), s)) != SCN_OK) return st;
  return launch_fwd<5>(b.act[4], blob, b.half, layer_geom(d, 5, n), s);
}

// Training forward: every activation is kept for the backward pass.
scn_status net_forward(const NetDims& d, int64_t n, const uint8_t* blob, const NetBuffers& b, hipStream_t s) {
  scn_status st;
  if ((st = launch_fwd<0>(b.x, blob, b.act[0], layer_geom(d, 0, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<1>(b.act[0], blob, b.act[1], layer_geom(d, 1, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<2>(b.act[1], blob, b.act[2], layer_geom(d, 2, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<3>(b.act[2], blob, b.act[3], layer_geom(d, 3, n), s)) != SCN_OK) return st;
  if ((st = launch_fwd<4>(b.act[3], blob, b.act[4], layer_geom(d, 4, n), s)) != SCN_OK) return st;
  return launch_fwd<5>(b.act[4], blob, b.half, layer_geom(d, 5, n), s);
}

scn_status dx_post(const float* dxe, const bf16_t* act, bf16_t* gout, const NetDims& d, int l_prev_out, int64_t n,
                   int up, hipStream_t s) {
  // l_prev_out: index of the stored activation (layer output l_prev_out) the gradient belongs to
  const int32_t h = d.hl[l_prev_out + 1], w = d.wl[l_prev_out + 1], c = kNet[l_prev_out].co;
  static_assert(kNet[0].co % 8 == 0 && kNet[1].co % 8 == 0 && kNet[2].co % 8 == 0 && kNet[3].co % 8 == 0 &&
                    kNet[4].co % 8 == 0,
                "k_dx_post takes 8 channels per thread");
  const int64_t groups = n * h * w * (c / 8);
  if ((groups + 255) / 256 > 0x7FFFFFFF) { set_error("surrogate batch too large"); return SCN_EUNSUPPORTED; }
  hipLaunchKernelGGL(k_dx_post, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, dxe, act, gout, groups, h, w,
                     c, up);
  SCN_LAUNCHED("input-gradient post launch");
  return SCN_OK;
}

scn_status net_backward(const NetDims& d, int64_t n, const uint8_t* blob, const NetBuffers& b, float* grads,
                        hipStream_t s) {
  scn_status st;
  // conv6: dy = ghalf (FP32), input act5
  if ((st = launch_dw<5>(b.ghalf, b.act[4], b, grads, layer_geom(d, 5, n), s)) != SCN_OK) return st;
  if ((st = launch_dx<5>(b.ghalf, blob, b.dxe, layer_geom(d, 5, n), s, b.act[4], b.g[0])) != SCN_OK) return st;
  // conv5: dy = g[0], input up(act4)
  if ((st = launch_dw<4>(b.g[0], b.act[3], b, grads, layer_geom(d, 4, n), s)) != SCN_OK) return st;
  if ((st = launch_dx<4>(b.g[0], blob, b.dxe, layer_geom(d, 4, n), s)) != SCN_OK) return st;
  if ((st = dx_post(b.dxe, b.act[3], b.g[1], d, 3, n, 1, s)) != SCN_OK) return st;
  // conv4: dy = g[1], input up(act3)
  if ((st = launch_dw<3>(b.g[1], b.act[2], b, grads, layer_geom(d, 3, n), s)) != SCN_OK) return st;
  if ((st = launch_dx<3>(b.g[1], blob, b.dxe, layer_geom(d, 3, n), s)) != SCN_OK) return st;
  if ((st = dx_post(b.dxe, b.act[2], b.g[0], d, 2, n, 1, s)) != SCN_OK) return st;
  // conv3: dy = g[0], input act2 (stride 2)
  if ((st = launch_dw<2>(b.g[0], b.act[1], b, grads, layer_geom(d, 2, n), s)) != SCN_OK) return st;
  if ((st = launch_dx<2>(b.g[0], blob, b.dxe, layer_geom(d, 2, n), s, b.act[1], b.g[1])) != SCN_OK) return st;
  // conv2: dy = g[1], input act1 (stride 2)
  if ((st = launch_dw<1>(b.g[1], b.act[0], b, grads, layer_geom(d, 1, n), s)) != SCN_OK) return st;
  if ((st = launch_dx<1>(b.g[1], blob, b.dxe, layer_geom(d, 1, n), s, b.act[0], b.g[0])) != SCN_OK) return st;
  // conv1: dy = g[0], input x
  return launch_dw<0>(b.g[0], b.x, b, grads, layer_geom(d, 0, n), s);
}

scn_status launch_net_input(const FrameDesc* frames, const PairDesc* pairs, bf16_t* x, const NetDims& d, int64_t n,
                            hipStream_t s) {
  const int64_t ne = n * d.h * d.w;
  hipLaunchKernelGGL(k_net_input, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, frames, pairs, x, d.h, d.w, n);
  SCN_LAUNCHED("network input launch");
  return SCN_OK;
}

scn_status launch_flow_up(const float* half, const PairDesc* pairs, const NetDims& d, int64_t n, hipStream_t s) {
  const int64_t ne = n * 4 * (int64_t)d.h * d.w;
  KernelTimer timer("flow_up", s);
  hipLaunchKernelGGL(k_flow_up, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, half, pairs, d.h, d.w, n);
  SCN_LAUNCHED("flow upsample launch");
  return SCN_OK;
}

scn_status launch_up_gate(const float* half, const FrameDesc* frames, const PairDesc* pairs, float* part,
                          const NetDims& d, int64_t n, float tau, uint8_t* active, hipStream_t s) {
  const int32_t W = 2 * d.w, H = 2 * d.h;
  const int32_t bpp = (int32_t)(((int64_t)(W / kGatePx) * H + 255) / 256);
  KernelTimer timer("gate", s);
  hipLaunchKernelGGL((k_up_gate<kGateGX, kGateGY>), dim3((unsigned)(bpp * n)), dim3(256), 0, s, half, frames, pairs, part, d.h,
                     d.w, bpp);
  SCN_LAUNCHED("upsample + gate launch");
  hipLaunchKernelGGL(k_gate_final, dim3((unsigned)n), dim3(256), 0, s, part, bpp,
                     1.f / ((float)W * H), tau, pairs, active);
  SCN_LAUNCHED("gate reduce launch");
  return SCN_OK;
}

size_t gate_part_bytes(int32_t W, int32_t H, int64_t n) {
  return align_up((size_t)n * (((size_t)W * H / kGatePx + 255) / 256 + 1) * 4);
}

}  // namespace sg

scn_status run_flow_chunk(const FlowPlan& plan, const FlowGroup& grp, const FlowChunk& ch,
                          const scn_flow_params& prm, void* ws, const uint8_t* active, const uint8_t* factive,
                          const int32_t* act_list, const int32_t* act_count, hipStream_t s, bool warm);

namespace {

const scn_flow_params kNoFlowParams = {1, 1.f, 0, 0, 0, 0};

size_t surrogate_extra(int32_t w, int32_t h) {
  const sg::NetLayout L = sg::net_layout(w, h, 1, false);
  return L.bytes + sg::gate_part_bytes(w, h, 1) + 2 * 256 + 32 * 256;
}

scn_status check_net_shape(const FlowPlan& plan) {
  for (const FlowGroup& g : plan.groups)
    if (g.w % 8 || g.h % 8) {
      set_error("the surrogate needs width and height that are multiples of 8");
      return SCN_EUNSUPPORTED;
    }
  return SCN_OK;
}

// grads / infer: every pair of the call in one batch of one resolution
scn_status batch_plan(const scn_job* jobs, int32_t n_jobs, float* const* outs, FlowPlan* plan, bool training,
                      size_t* need) {
  scn_status st = build_flow_plan(jobs, n_jobs, &kNoFlowParams, outs, 0, plan);
  if (st != SCN_OK) return st;
  if (plan->groups.size() > 1) {
    set_error("surrogate training and inference batches need one resolution");
    return SCN_EUNSUPPORTED;
  }
  if ((st = check_net_shape(*plan)) != SCN_OK) return st;
  *need = plan->scratch_off;
  if (!plan->groups.empty())
    *need += sg::net_layout(plan->groups[0].w, plan->groups[0].h, plan->groups[0].total_pairs, training).bytes;
  return SCN_OK;
}

}  // namespace

size_t surrogate_ws_bytes(int32_t op, const scn_job* jobs, int32_t n_jobs, const scn_flow_params* p) {
  FlowPlan plan;
  size_t need = 0;
  if (op == SCN_OP_SURROGATE) {
    if (build_flow_plan(jobs, n_jobs, p, nullptr, 0, &plan, surrogate_extra) != SCN_OK) return 0;
    if (check_net_shape(plan) != SCN_OK) return 0;
    return plan.ws_needed;
  }
  if (batch_plan(jobs, n_jobs, nullptr, &plan, op == SCN_OP_SURROGATE_GRADS, &need) != SCN_OK) return 0;
  return need;
}

}  // namespace scn

using namespace scn;

extern "C" {

size_t scn_net_bytes(void) { return (size_t)sg::kBlobBytes; }

int32_t scn_net_params(void) { return sg::kParams; }

scn_status scn_net_pack(const float* master, void* net, scn_stream_t stream) {
  clear_error();
  if (!master || !net) { set_error("NULL argument"); return SCN_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  const int64_t words = sg::kBlobBytes / 4;
  hipLaunchKernelGGL(sg::k_zero_bytes, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (uint32_t*)net, words);
  SCN_LAUNCHED("net zero launch");
  hipLaunchKernelGGL(sg::k_pack, dim3((sg::kParams + 255) / 256), dim3(256), 0, s, master, (uint8_t*)net);
  SCN_LAUNCHED("net pack launch");
  return SCN_OK;
}

scn_status scn_adam_step(float* master, float* m, float* v, const float* grads, int32_t step, float lr, float beta1,
                         float beta2, float eps, void* net, scn_stream_t stream) {
  clear_error();
  if (!master || !m || !v || !grads || !net) { set_error("NULL argument"); return SCN_EINVAL; }
  if (step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
    set_error("bad Adam hyper-parameters");
    return SCN_EINVAL;
  }
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipLaunchKernelGGL(sg::k_adam, dim3((sg::kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, master, m, v,
                     grads, lr, beta1, beta2, eps, bc1, bc2, (uint8_t*)net);
  SCN_LAUNCHED("adam launch");
  return SCN_OK;
}

scn_status scn_surrogate_grads(const scn_job* jobs, int32_t n_jobs, const void* net, float* const* targets,
                               float* grads, float* loss, void* ws, size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  FlowPlan plan;
  size_t need = 0;
  scn_status st = batch_plan(jobs, n_jobs, targets, &plan, true, &need);
  if (st != SCN_OK) return st;
  if (plan.total_pairs == 0) { set_error("no pairs"); return SCN_EINVAL; }
  if (!net || !grads || !loss || !ws) { set_error("NULL argument"); return SCN_EINVAL; }
  if (ws_bytes < need) { set_error("workspace too small for surrogate gradients"); return SCN_ENOSPACE; }
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_plan(ws, plan.plan_bytes.data(), plan.plan_bytes.size(), s)) != SCN_OK) return st;
  const FlowGroup& grp = plan.groups[0];
  const FlowChunk& ch = grp.chunks[0];
  uint8_t* base = (uint8_t*)ws;
  const sg::NetLayout L = sg::net_layout(grp.w, grp.h, ch.n_pairs, true);
  const sg::NetBuffers b = sg::net_buffers(base + plan.scratch_off, L, true);
  const sg::NetDims d = sg::net_dims(grp.w, grp.h);
  const FrameDesc* frames = (const FrameDesc*)(base + ch.frames_off);
  const PairDesc* pairs = (const PairDesc*)(base + ch.pairs_off);
  const uint8_t* blob = (const uint8_t*)net;
  const int64_t n = ch.n_pairs;
  if ((st = sg::launch_net_input(frames, pairs, b.x, d, n, s)) != SCN_OK) return st;
  if ((st = sg::net_forward(d, n, blob, b, s)) != SCN_OK) return st;
  const int64_t nh = n * d.h * d.w;
  const int64_t blocks = (nh + 255) / 256;
  const float scale = 1.f / ((float)grp.w * grp.h * (float)n);
  hipLaunchKernelGGL(sg::k_loss_grad, dim3((unsigned)blocks), dim3(256), 0, s, b.half, pairs, b.ghalf, b.loss_part,
                     d.h, d.w, n, scale);
  SCN_LAUNCHED("loss launch");
  hipLaunchKernelGGL(sg::k_sum_loss, dim3(1), dim3(256), 0, s, b.loss_part, blocks, scale, loss);
  SCN_LAUNCHED("loss reduce launch");
  return sg::net_backward(d, n, blob, b, grads, s);
}

scn_status scn_surrogate_train_step(const scn_job* jobs, int32_t n_jobs, float* const* targets, float* master,
                                    float* m, float* v, float* grads, void* net, int32_t step, float lr, float beta1,
                                    float beta2, float eps, float* loss, void* ws, size_t ws_bytes,
                                    scn_stream_t stream) {
  clear_error();
  // the Adam part's arguments first: the gradient part enqueues as soon as
  // its own arguments check out
  if (!master || !m || !v || !grads || !net) { set_error("NULL argument"); return SCN_EINVAL; }
  if (step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
    set_error("bad Adam hyper-parameters");
    return SCN_EINVAL;
  }
  scn_status st = scn_surrogate_grads(jobs, n_jobs, net, targets, grads, loss, ws, ws_bytes, stream);
  if (st != SCN_OK) return st;
  return scn_adam_step(master, m, v, grads, step, lr, beta1, beta2, eps, net, stream);
}

scn_status scn_surrogate_infer(const scn_job* jobs, int32_t n_jobs, const void* net, float* const* flow, void* ws,
                               size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  FlowPlan plan;
  size_t need = 0;
  scn_status st = batch_plan(jobs, n_jobs, flow, &plan, false, &need);
  if (st != SCN_OK) return st;
  if (plan.total_pairs == 0) return SCN_OK;
  if (!net || !ws) { set_error("NULL argument"); return SCN_EINVAL; }
  if (ws_bytes < need) { set_error("workspace too small for surrogate inference"); return SCN_ENOSPACE; }
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_plan(ws, plan.plan_bytes.data(), plan.plan_bytes.size(), s)) != SCN_OK) return st;
  const FlowGroup& grp = plan.groups[0];
  const FlowChunk& ch = grp.chunks[0];
  uint8_t* base = (uint8_t*)ws;
  const sg::NetLayout L = sg::net_layout(grp.w, grp.h, ch.n_pairs, false);
  const sg::NetBuffers b = sg::net_buffers(base + plan.scratch_off, L, false);
  const sg::NetDims d = sg::net_dims(grp.w, grp.h);
  const FrameDesc* frames = (const FrameDesc*)(base + ch.frames_off);
  const PairDesc* pairs = (const PairDesc*)(base + ch.pairs_off);
  if ((st = sg::net_forward_infer(frames, pairs, d, ch.n_pairs, (const uint8_t*)net, b, s)) != SCN_OK) return st;
  return sg::launch_flow_up(b.half, pairs, d, ch.n_pairs, s);
}

scn_status scn_flow_surrogate(const scn_job* jobs, int32_t n_jobs, const scn_flow_params* fallback_p, const void* net,
                              float gate_tau, float* const* flow, uint8_t* const* fell_back, float* const* residual,
                              void* ws, size_t ws_bytes, scn_stream_t stream) {
  clear_error();
  FlowPlan plan;
  scn_status st = build_flow_plan(jobs, n_jobs, fallback_p, flow, ws_bytes, &plan, surrogate_extra, fell_back,
                                  residual);
  if (st != SCN_OK) return st;
  if ((st = check_net_shape(plan)) != SCN_OK) return st;
  if (plan.total_pairs == 0) return SCN_OK;
  if (!net || !ws) { set_error("NULL argument"); return SCN_EINVAL; }
  if (!(gate_tau >= 0.f)) { set_error("gate_tau must be >= 0"); return SCN_EINVAL; }
  if (ws_bytes < plan.ws_min) { set_error("workspace too small for the surrogate path"); return SCN_ENOSPACE; }
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_plan(ws, plan.plan_bytes.data(), plan.plan_bytes.size(), s)) != SCN_OK) return st;
  uint8_t* base = (uint8_t*)ws;
  for (const FlowGroup& grp : plan.groups) {
    const sg::NetDims d = sg::net_dims(grp.w, grp.h);
    for (const FlowChunk& ch : grp.chunks) {
      const int64_t n = ch.n_pairs;
      uint8_t* extra = base + plan.scratch_off + chunk_pyr_bytes(grp, ch) + chunk_pairs_bytes(grp, ch);
      const sg::NetLayout L = sg::net_layout(grp.w, grp.h, n, false);
      const sg::NetBuffers b = sg::net_buffers(extra, L, false);
      float* gpart = (float*)(extra + L.bytes);
      uint8_t* active = extra + L.bytes + sg::gate_part_bytes(grp.w, grp.h, n);
      uint8_t* factive = active + align_up((size_t)n);
      const FrameDesc* frames = (const FrameDesc*)(base + ch.frames_off);
      const PairDesc* pairs = (const PairDesc*)(base + ch.pairs_off);
      if ((st = sg::net_forward_infer(frames, pairs, d, n, (const uint8_t*)net, b, s)) != SCN_OK) return st;
      if ((st = sg::launch_up_gate(b.half, frames, pairs, gpart, d, n, gate_tau, active, s)) != SCN_OK) return st;
      const int64_t fw = (ch.n_frames + 3) / 4;
      hipLaunchKernelGGL(sg::k_zero_bytes, dim3((unsigned)((fw + 255) / 256)), dim3(256), 0, s, (uint32_t*)factive,
                         fw);
      hipLaunchKernelGGL(sg::k_mark_frames, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pairs, active,
                         factive, n);
      int32_t* act_list = (int32_t*)(factive + align_up((size_t)ch.n_frames));
      int32_t* act_count = act_list + align_up((size_t)n);
      hipLaunchKernelGGL(sg::k_compact_active, dim3(1), dim3(256), 0, s, active, n, act_list, act_count);
      SCN_LAUNCHED("fallback frame marking launch");
      if ((st = run_flow_chunk(plan, grp, ch, *fallback_p, ws, active, factive, act_list, act_count, s, false)) !=
          SCN_OK)
        return st;
    }
  }
  return SCN_OK;
}

}  // extern "C"
