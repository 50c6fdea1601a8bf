// Pyramidal Horn-Schunck optical flow (Horn & Schunck 1981) between
// consecutive sampled frames -- the FLOW stencil S[0,1] of the Scanner paper
// (Sec. 3.2, Sec. 5.1.2) -- for gfx950, FP32.
//
// Per pair and pyramid level (coarse to fine), in one setup kernel:
//   warp:  u0, v0 = 2 * bilinear(coarser flow, x/2, y/2) (zero at the coarsest
//          level); T = bilinear(I2, x + u0, y + v0), coordinates clamped.
//   coef:  Ix = (Dx I1 + Dx T)/2, Iy likewise (central differences,
//          clamp-to-edge), It' = (T - I1) - Ix u0 - Iy v0;
//          with r = 1/sqrt(alpha^2 + Ix^2 + Iy^2) the kernel stores
//          a = Ix r, b = Iy r, c = It' r, so that the Jacobi update
//          u <- ubar - Ix (Ix ubar + Iy vbar + It') / (alpha^2 + Ix^2 + Iy^2)
//          becomes u <- ubar - a s, v <- vbar - b s with s = a ubar + b vbar + c.
//   jacobi: ubar = (sum of edge neighbours)/6 + (sum of diagonals)/12 with
//          clamp-to-edge, written as ubar = (cu(x-1) + cu(x+1) + 2 p(x)) / 12
//          where p(x) = u(x, y-1) + u(x, y+1) and cu(x) = 2 u(x, y) + p(x).
//
// Every Jacobi kernel evaluates exactly that sequence of FP32 operations per
// pixel (explicit fmaf, no contraction), so all of them -- one sweep per
// launch, or several sweeps per launch on register/LDS tiles with mirrored
// halos -- produce bitwise identical flow.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "flow_plan.hpp"

namespace scn {

namespace {

constexpr int kThreads = 256;

struct LevelGeom {
  int32_t w, h;        // this level
  int32_t cw, ch;      // coarser level (valid when has_coarse)
  int32_t has_coarse;
  int64_t n0;          // level-0 pixels (plane stride inside a pair's scratch)
  int64_t lvl_off;     // float offset of this level inside a pyramid slot (l >= 1; stored as doubles)
  int32_t level;
};

struct ChunkPtrs {
  const FrameDesc* frames;
  const PairDesc* pairs;
  float* pyr;            // pyramid slots, pyr_floats each
  int64_t pyr_floats;
  float* scratch;        // pair scratch, pair_floats each
  int64_t pair_floats;
  int64_t n_pairs, n_frames;
  const uint8_t* active;   // per pair: compute this pair (NULL: all pairs)
  const uint8_t* factive;  // per frame: some active pair uses it (NULL: all frames)
  // with a mask: the active pairs in ascending order and their count (device);
  // the streaming Jacobi walks this list instead of every pair
  const int32_t* act_list;
  const int32_t* act_count;
};

// Every buffer the kernels touch is device global memory.  Pointers read
// from the descriptor tables would otherwise be generic (flat) pointers,
// whose accesses also count against the LDS wait counter and need 64-bit
// per-lane address arithmetic; passing them through the global address
// space lets the compiler emit global accesses.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)p;
}
// Load of a global element at a (wave-uniform) base plus a 32-bit byte
// offset: a scalar base and one VGPR offset, no per-lane 64-bit arithmetic.
// The base is converted to a global pointer before the offset is added, so
// that the sum is a global-address-space sum (scalar base + 32-bit vector
// offset in one instruction) rather than a 64-bit generic sum per lane.
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) const char gcchar;
template <typename T>
__device__ __forceinline__ T ldg(const T* base, uint32_t byte_off) {
  return *(const __attribute__((address_space(1))) T*)((gcchar*)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void stg(T* base, uint32_t byte_off, T v) {
  *(__attribute__((address_space(1))) T*)((gchar*)base + byte_off) = v;
}

// (u, v) buffer codes: 0 and 1 are the pair's ping-pong buffers, 2 is the output.
__device__ __forceinline__ float* uv_buf(const ChunkPtrs& c, int64_t pair, int code, int64_t n0) {
  if (code == 2) return as_global(c.pairs[pair].out);
  return as_global(c.scratch + pair * c.pair_floats + (int64_t)(kPlaneU0 + 2 * code) * n0);
}
__device__ __forceinline__ float* plane(const ChunkPtrs& c, int64_t pair, int k, int64_t n0) {
  return as_global(c.scratch + pair * c.pair_floats + (int64_t)k * n0);
}

// Image of level l of frame slot f: u8 luma at level 0, the exact pyramid
// (FP64) above.
struct Img {
  const uint8_t* y8;
  const double* f;
  int64_t pitch;
};
__device__ __forceinline__ Img level_img(const ChunkPtrs& c, int32_t f, const LevelGeom& g) {
  Img im;
  if (g.level == 0) {
    im.y8 = as_global(c.frames[f].y);
    im.f = nullptr;
    im.pitch = c.frames[f].pitch;
  } else {
    im.y8 = nullptr;
    im.f = as_global(reinterpret_cast<const double*>(c.pyr + (int64_t)f * c.pyr_floats + g.lvl_off));
    im.pitch = g.w;
  }
  return im;
}

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return min(max(v, lo), hi); }

// ---------------------------------------------------------------------------
// pyramid: level l = even samples of blur5(level l-1), [1,4,6,4,1]/16
// horizontal then vertical, clamp-to-edge.  A workgroup owns 16 x 64 output
// pixels: it stages the 35 x 131 clamped input pixels in LDS with coalesced
// loads, forms the horizontal sums of the 35 rows at the 64 even columns, and
// then the vertical sums.  The levels are exact: a level-l value is an integer
// multiple of 2^-8l below 256 (8 + 8l significant bits), so integer sums at
// level 0 and FP64 sums above (53-bit significand) round nothing through
// level 5, and the stored FP64 values equal the plain definition's.  (Levels
// rounded to FP32 at every step move the flow of ill-conditioned pixels --
// occlusion edges under large displacements -- by several 1e-3 px.)
constexpr int kPyrTW = 64, kPyrTH = 16, kPyrIW = 2 * kPyrTW + 3, kPyrIH = 2 * kPyrTH + 3;
template <bool U8>
__global__ void __launch_bounds__(256) k_pyr_down(ChunkPtrs c, LevelGeom src, LevelGeom dst, int32_t tiles_x,
                                                  int32_t tiles_per_frame) {
  using T = typename std::conditional<U8, int, double>::type;
  __shared__ __attribute__((aligned(16))) T sIn[kPyrIH][kPyrIW + 1];
  __shared__ T sH[kPyrIH][kPyrTW];
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t f = blk / tiles_per_frame;
  if (c.factive && !c.factive[f]) return;
  const int32_t t = blk % tiles_per_frame;
  const int32_t ox = (t % tiles_x) * kPyrTW, oy = (t / tiles_x) * kPyrTH;
  const int32_t ix0 = 2 * ox - 2, iy0 = 2 * oy - 2;
  const Img im = level_img(c, (int32_t)f, src);
  constexpr int NIN = kPyrIH * kPyrIW, IT = (NIN + 255) / 256;
  // Level 0 tiles whose input lies inside the frame read their 35 rows as
  // 33 four-byte words each (unaligned global loads are allowed; the 132nd
  // byte lands in the row's padding column), the others byte by byte with
  // clamped coordinates.
  const bool words = U8 && ix0 >= 0 && ix0 + 4 * (kPyrIW / 4 + 1) <= src.w && iy0 >= 0 && iy0 + kPyrIH <= src.h;
  if constexpr (U8) {
    if (words) {
      constexpr int WPR = kPyrIW / 4 + 1, NW = kPyrIH * WPR, ITW = (NW + 255) / 256;
      uint32_t wv[ITW];
#pragma unroll
      for (int i = 0; i < ITW; ++i) {
        const int e = min((int)threadIdx.x + i * 256, NW - 1);
        const uint32_t off = (uint32_t)(iy0 + e / WPR) * (uint32_t)im.pitch + (uint32_t)(ix0 + 4 * (e % WPR));
        wv[i] = ldg(reinterpret_cast<const uint32_t*>(im.y8), off);
      }
#pragma unroll
      for (int i = 0; i < ITW; ++i) {
        const int e = threadIdx.x + i * 256;
        if (e < NW)
          *reinterpret_cast<int4*>(&sIn[e / WPR][4 * (e % WPR)]) =
              make_int4((int)(wv[i] & 0xFFu), (int)((wv[i] >> 8) & 0xFFu), (int)((wv[i] >> 16) & 0xFFu),
                        (int)(wv[i] >> 24));
      }
    }
  }
  if (!words) {
    T v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = min((int)threadIdx.x + i * 256, NIN - 1);
      const int32_t yy = clampi(iy0 + e / kPyrIW, 0, src.h - 1), xx = clampi(ix0 + e % kPyrIW, 0, src.w - 1);
      const uint32_t off = (uint32_t)yy * (uint32_t)im.pitch + (uint32_t)xx;
      if constexpr (U8) v[i] = (int)ldg(im.y8, off);
      else v[i] = ldg(im.f, 8u * off);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = threadIdx.x + i * 256;
      if (e < NIN) sIn[e / kPyrIW][e % kPyrIW] = v[i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kPyrIH * kPyrTW; e += 256) {
    const int r = e / kPyrTW, x = e % kPyrTW;
    if constexpr (U8) {
      const int ki[5] = {1, 4, 6, 4, 1};
      int hs = 0;
#pragma unroll
      for (int i = 0; i < 5; ++i) hs += ki[i] * sIn[r][2 * x + i];
      sH[r][x] = hs;
    } else {
      const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
      double hs = 0.0;
#pragma unroll
      for (int i = 0; i < 5; ++i) hs += k[i] * sIn[r][2 * x + i];
      sH[r][x] = hs;
    }
  }
  __syncthreads();
  double* out = reinterpret_cast<double*>(c.pyr + f * c.pyr_floats + dst.lvl_off);
  for (int e = threadIdx.x; e < kPyrTH * kPyrTW; e += 256) {
    const int ly = e / kPyrTW, x = e % kPyrTW;
    const int32_t gx = ox + x, gy = oy + ly;
    if (gx >= dst.w || gy >= dst.h) continue;
    double acc;
    if constexpr (U8) {
      const int ki[5] = {1, 4, 6, 4, 1};
      int s = 0;
#pragma unroll
      for (int j = 0; j < 5; ++j) s += ki[j] * sH[2 * ly + j][x];
      acc = (double)s * (1.0 / 256.0);
    } else {
      const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
      acc = 0.0;
#pragma unroll
      for (int j = 0; j < 5; ++j) acc += k[j] * sH[2 * ly + j][x];
    }
    stg(out, 8u * ((uint32_t)gy * (uint32_t)dst.w + (uint32_t)gx), acc);
  }
}

// setup = warp + coef fused on 64 x 16 output tiles: the warped image T, the
// start flow and I1 of the tile plus a one-pixel clamped halo go to LDS, then
// the gradients and coefficients use the same expressions as k_hs_warp and
// k_hs_coef (so the results are bitwise identical) without the T round trip
// through HBM.
constexpr int kSetupTW = 64, kSetupTH = 16;
// U8: level 0 (luma read as u8 from the table); COARSE: a coarser level
// exists (start flow from it).  Each thread gathers all of its halo-tile
// samples into registers before the first LDS store, so the loads of one
// thread overlap instead of waiting one by one.  Above level 0 the warp, the
// gradients and the linearised constraint are evaluated in FP64 on the exact
// pyramid (the coefficients are rounded to FP32 once): at level 0 the u8
// images are exact and FP32 suffices, while rounding the coarse levels'
// images and gradients moves ill-conditioned pixels by up to 1e-3 px.
template <bool U8, bool COARSE, bool INIT, bool LIST>
__global__ void __launch_bounds__(256) k_hs_setup(ChunkPtrs c, LevelGeom g, int32_t coarse_code, int32_t dst_code,
                                                  float alpha2, int32_t tiles_x, int32_t tiles_per_pair) {
  using T = typename std::conditional<U8, float, double>::type;  // arithmetic of warp and gradients
  constexpr int TW = kSetupTW + 2, NE = (kSetupTH + 2) * TW, IT = (NE + 255) / 256;
  __shared__ T sT[kSetupTH + 2][kSetupTW + 2];
  __shared__ T sI[kSetupTH + 2][kSetupTW + 2];
  __shared__ float sU[kSetupTH][kSetupTW];
  __shared__ float sV[kSetupTH][kSetupTW];
  // A workgroup takes tile `unit` = its index; with an active-pair list (a
  // masked solve) the units index list slots and the grid, sized for a
  // fraction of the pairs, strides over them until the list is exhausted.
  // (units stay below 2^31: the host bounds tiles x pairs)
  for (uint32_t unit = xcd_block(blockIdx.x, gridDim.x);; unit += gridDim.x) {
    int64_t pr;
    const uint32_t slot = unit / (uint32_t)tiles_per_pair;
    if constexpr (LIST) {
      if ((int64_t)slot >= *c.act_count) return;
      pr = c.act_list[slot];
    } else {
      pr = slot;
      if (c.active && !c.active[pr]) return;
    }
    const int32_t t = (int32_t)(unit % (uint32_t)tiles_per_pair);
    const int32_t ox = (t % tiles_x) * kSetupTW, oy = (t / tiles_x) * kSetupTH;
    const PairDesc pd = c.pairs[pr];
    const float* init_u = INIT ? as_global(pd.init) : nullptr;
    const float* init_v = INIT ? init_u + (int64_t)g.w * g.h : nullptr;
    const uint8_t* y1 = nullptr;
    const uint8_t* y2 = nullptr;
    const double* f1 = nullptr;
    const double* f2 = nullptr;
    int64_t p1, p2;
    if constexpr (U8) {
      const FrameDesc d1 = c.frames[pd.f1], d2 = c.frames[pd.f2];
      y1 = as_global(d1.y);
      y2 = as_global(d2.y);
      p1 = d1.pitch;
      p2 = d2.pitch;
    } else {
      f1 = as_global(reinterpret_cast<const double*>(c.pyr + (int64_t)pd.f1 * c.pyr_floats + g.lvl_off));
      f2 = as_global(reinterpret_cast<const double*>(c.pyr + (int64_t)pd.f2 * c.pyr_floats + g.lvl_off));
      p1 = p2 = g.w;
    }
    // 32-bit byte offsets (a frame or pyramid level is far below 4 GiB)
    const uint32_t q1 = (uint32_t)p1, q2 = (uint32_t)p2;
    // rows < 2^15 and pitches <= 2^20 (checked on the host): 24-bit products
    auto at1 = [&](int32_t xx, int32_t yy) -> T {
      if constexpr (U8) return (float)ldg(y1, __umul24((uint32_t)yy, q1) + (uint32_t)xx);
      else return ldg(f1, 8u * (__umul24((uint32_t)yy, q1) + (uint32_t)xx));
    };
    // Warped I2 at (X, Y) = (xi + xf, yi + yf), X given as integer + fraction
    // (exact far from the origin), clamped bilinear: outside [0, w-2] the x
    // fraction is 0 at the clamped column (likewise in y).  The two columns of
    // a row are read by one load (2 bytes at level 0, 8 bytes above; unaligned
    // global loads are allowed; 16-byte pairs of doubles above level 0) at
    // xs = clamp(xi, 0, w - 2); past the right edge the clamped sample is the
    // second element with weight 1, which is the same value as the clamped
    // column with weight 0.
    auto warp_sample = [&](int32_t xi, float xf, int32_t yi, float yf) -> T {
      int32_t xs;
      T fx;
      if (xi < 0) { xs = 0; fx = 0.f; } else if (xi >= g.w - 1) { xs = g.w - 2; fx = 1.f; } else { xs = xi; fx = xf; }
      const bool iny = (uint32_t)yi < (uint32_t)(g.h - 1);
      const int32_t y0 = clampi(yi, 0, g.h - 1), y1 = y0 + (iny ? 1 : 0);
      const T fy = iny ? yf : 0.f;
      T a0, b0, a1, b1;
      if constexpr (U8) {
        const uint32_t w0 = ldg(reinterpret_cast<const uint16_t*>(y2), __umul24((uint32_t)y0, q2) + (uint32_t)xs);
        const uint32_t w1 = ldg(reinterpret_cast<const uint16_t*>(y2), __umul24((uint32_t)y1, q2) + (uint32_t)xs);
        a0 = (float)(w0 & 0xFFu);
        b0 = (float)(w0 >> 8);
        a1 = (float)(w1 & 0xFFu);
        b1 = (float)(w1 >> 8);
      } else {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v r0 = ldg(reinterpret_cast<const d2v*>(f2), 8u * (__umul24((uint32_t)y0, q2) + (uint32_t)xs));
        const d2v r1 = ldg(reinterpret_cast<const d2v*>(f2), 8u * (__umul24((uint32_t)y1, q2) + (uint32_t)xs));
        a0 = r0.x;
        b0 = r0.y;
        a1 = r1.x;
        b1 = r1.y;
      }
      const T one = 1;
      const T top = (one - fx) * a0 + fx * b0;
      const T bot = (one - fx) * a1 + fx * b1;
      return (one - fy) * top + fy * bot;
    };
    // Start flow = 2 * bilinear(coarse flow, x/2, y/2), separably: the
    // horizontal interpolation of the coarse rows under the tile ((oy-1)/2 ..
    // (oy+16)/2 + 1, at most 11, clamped to the coarse level) at each of the
    // tile's 66 halo columns goes to LDS once; each halo pixel then combines
    // two of those rows.  Same operands and operation order as the plain
    // bilinear formula, so the values are identical.
    constexpr int CH = kSetupTH / 2 + 3;
    __shared__ float sHU[COARSE ? CH : 1][COARSE ? TW : 1];
    __shared__ float sHV[COARSE ? CH : 1][COARSE ? TW : 1];
    int32_t cy_lo = 0;
    if constexpr (COARSE) {
      const float* cu = uv_buf(c, pr, coarse_code, g.n0);
      const float* cv = cu + (int64_t)g.cw * g.ch;
      cy_lo = min(max(oy - 1, 0) >> 1, g.ch - 1);
      constexpr int NH = CH * TW, ITH = (NH + 255) / 256;
      const uint32_t cw4 = 4u * (uint32_t)g.cw;
      float ha[ITH], hb[ITH], hc[ITH], hd[ITH], hf[ITH];
  #pragma unroll
      for (int i = 0; i < ITH; ++i) {
        const int e = min((int)threadIdx.x + i * 256, NH - 1);
        const int32_t yy = min(cy_lo + e / TW, g.ch - 1);
        const int32_t x = clampi(ox + e % TW - 1, 0, g.w - 1), xi = x >> 1;
        int32_t x0;
        if (xi >= g.cw - 1) { x0 = g.cw - 1; hf[i] = 0.f; }
        else { x0 = xi; hf[i] = (x & 1) ? 0.5f : 0.f; }
        const int32_t x1 = min(x0 + 1, g.cw - 1);
        const uint32_t r = __umul24((uint32_t)yy, cw4);
        ha[i] = ldg(cu, r + 4u * (uint32_t)x0);
        hb[i] = ldg(cu, r + 4u * (uint32_t)x1);
        hc[i] = ldg(cv, r + 4u * (uint32_t)x0);
        hd[i] = ldg(cv, r + 4u * (uint32_t)x1);
      }
  #pragma unroll
      for (int i = 0; i < ITH; ++i) {
        const int e = threadIdx.x + i * 256;
        if (e < NH) {
          const float fx = hf[i];
          sHU[e / TW][e % TW] = (1.f - fx) * ha[i] + fx * hb[i];
          sHV[e / TW][e % TW] = (1.f - fx) * hc[i] + fx * hd[i];
        }
      }
      __syncthreads();
    }
    T rT[IT], rI[IT];
    float rU[IT], rV[IT];
    // halo element e = tid + 256 i at (ty, tx) = (e / TW, e % TW), advanced
    // incrementally (256 = 3 TW + 58); elements past the tile repeat the last
    int hty = (int)threadIdx.x / TW, htx = (int)threadIdx.x % TW;
  #pragma unroll
    for (int i = 0; i < IT; ++i) {
      if (i > 0) {
        htx += 256 % TW;
        hty += 256 / TW;
        if (htx >= TW) { htx -= TW; ++hty; }
      }
      const bool past = hty >= kSetupTH + 2;
      const int ty = past ? kSetupTH + 1 : hty, tx = past ? TW - 1 : htx;
      const int32_t x = clampi(ox + tx - 1, 0, g.w - 1), y = clampi(oy + ty - 1, 0, g.h - 1);
      float u0 = 0.f, v0 = 0.f;
      if constexpr (INIT) {
        // warm start: the predecessor pair's full-resolution flow
        const uint32_t o = 4u * (__umul24((uint32_t)y, (uint32_t)g.w) + (uint32_t)x);
        u0 = ldg(init_u, o);
        v0 = ldg(init_v, o);
      }
      if constexpr (COARSE) {
        const int32_t yi = y >> 1;
        int32_t y0;
        float fy;
        if (yi >= g.ch - 1) { y0 = g.ch - 1; fy = 0.f; }
        else { y0 = yi; fy = (y & 1) ? 0.5f : 0.f; }
        const int r0 = y0 - cy_lo, r1 = min(y0 + 1, g.ch - 1) - cy_lo;
        u0 = 2.f * ((1.f - fy) * sHU[r0][tx] + fy * sHU[r1][tx]);
        v0 = 2.f * ((1.f - fy) * sHV[r0][tx] + fy * sHV[r1][tx]);
      }
      const float fu = floorf(u0), fv = floorf(v0);
      rT[i] = warp_sample(x + (int32_t)fu, u0 - fu, y + (int32_t)fv, v0 - fv);
      rI[i] = at1(x, y);
      rU[i] = u0;
      rV[i] = v0;
    }
  #pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int e = threadIdx.x + i * 256;
      if (e >= NE) break;
      const int ty = e / TW, tx = e % TW;
      sT[ty][tx] = rT[i];
      sI[ty][tx] = rI[i];
      const int iy = ty - 1, ix = tx - 1;
      if (iy >= 0 && iy < kSetupTH && ix >= 0 && ix < kSetupTW) {
        sU[iy][ix] = rU[i];
        sV[iy][ix] = rV[i];
      }
    }
    __syncthreads();
    const int64_t n = (int64_t)g.w * g.h;
    float* pa = plane(c, pr, kPlaneA, g.n0);
    float* pb = plane(c, pr, kPlaneB, g.n0);
    float* pc = plane(c, pr, kPlaneC, g.n0);
    float* dst = uv_buf(c, pr, dst_code, g.n0);
    for (int e = threadIdx.x; e < kSetupTH * kSetupTW; e += 256) {
      const int ly = e / kSetupTW, lx = e % kSetupTW;
      const int32_t x = ox + lx, y = oy + ly;
      if (x >= g.w || y >= g.h) continue;
      const int hx = lx + 1, hy = ly + 1;
      // clamp-to-edge neighbours: the halo holds the clamped pixels, and at the
      // image's own border the neighbour index is clamped onto the pixel itself
      const int xl = (x > 0) ? hx - 1 : hx, xr = (x < g.w - 1) ? hx + 1 : hx;
      const int yu = (y > 0) ? hy - 1 : hy, yd = (y < g.h - 1) ? hy + 1 : hy;
      const float u0 = sU[ly][lx], v0 = sV[ly][lx];
      // Ix = (central difference of I1 + that of T) / 2 with each difference
      // halved: the two power-of-two scalings are folded into one factor 1/4
      // (exact: scaling by 2^-k commutes with rounding for these magnitudes)
      const T Ix = ((sI[hy][xr] - sI[hy][xl]) + (sT[hy][xr] - sT[hy][xl])) * (T)0.25;
      const T Iy = ((sI[yd][hx] - sI[yu][hx]) + (sT[yd][hx] - sT[yu][hx])) * (T)0.25;
      const T It = sT[hy][hx] - sI[hy][hx];
      const T Itp = It - Ix * (T)u0 - Iy * (T)v0;
      const T den = (T)alpha2 + Ix * Ix + Iy * Iy;
      T r;
      if constexpr (U8) r = rsqrtf(den);  // within a few ulps; den >= alpha^2 > 0
      else r = 1.0 / sqrt(den);
      const uint32_t p4 = 4u * (__umul24((uint32_t)y, (uint32_t)g.w) + (uint32_t)x);
      stg(pa, p4, (float)(Ix * r));
      stg(pb, p4, (float)(Iy * r));
      stg(pc, p4, (float)(Itp * r));
      stg(dst, p4, u0);
      stg(dst, p4 + 4u * (uint32_t)n, v0);
    }
    if constexpr (!LIST) return;  // one tile per workgroup without a list
    __syncthreads();              // the next tile reuses the LDS arrays
  }
}

// The per-pixel Jacobi update shared by every Jacobi kernel.
//   pu = u(x, y-1) + u(x, y+1); cl, cr = cu(x-1), cu(x+1) with cu = fma(u, 2, p).
__device__ __forceinline__ float jac_bar(float pu, float cl, float cr) {
  const float h = cl + cr;
  return __fmul_rn(fmaf(pu, 2.f, h), 1.f / 12.f);
}
__device__ __forceinline__ float jac_col(float up, float mid, float dn) { return fmaf(mid, 2.f, up + dn); }
__device__ __forceinline__ void jac_update(float ub, float vb, float a, float b, float c, float* u, float* v) {
  const float s = fmaf(a, ub, fmaf(b, vb, c));
  *u = fmaf(-a, s, ub);
  *v = fmaf(-b, s, vb);
}

// One Jacobi sweep, one thread per pixel (reference kernel, global reads).
__global__ void __launch_bounds__(kThreads) k_hs_jacobi1(ChunkPtrs c, LevelGeom g, int32_t src_code, int32_t dst_code,
                                                         int32_t bpp) {
  const int64_t pr = blockIdx.x / bpp;
  const int64_t p = (int64_t)(blockIdx.x % bpp) * kThreads + threadIdx.x;
  const int64_t n = (int64_t)g.w * g.h;
  if (p >= n) return;
  if (c.active && !c.active[pr]) return;
  const int32_t x = (int32_t)(p % g.w), y = (int32_t)(p / g.w);
  const float* su = uv_buf(c, pr, src_code, g.n0);
  const float* sv = su + n;
  const int32_t xl = max(x - 1, 0), xr = min(x + 1, g.w - 1);
  const int64_t ru = (int64_t)max(y - 1, 0) * g.w, rm = (int64_t)y * g.w, rd = (int64_t)min(y + 1, g.h - 1) * g.w;
  const float ub = jac_bar(su[ru + x] + su[rd + x], jac_col(su[ru + xl], su[rm + xl], su[rd + xl]),
                           jac_col(su[ru + xr], su[rm + xr], su[rd + xr]));
  const float vb = jac_bar(sv[ru + x] + sv[rd + x], jac_col(sv[ru + xl], sv[rm + xl], sv[rd + xl]),
                           jac_col(sv[ru + xr], sv[rm + xr], sv[rd + xr]));
  float un, vn;
  jac_update(ub, vb, plane(c, pr, kPlaneA, g.n0)[p], plane(c, pr, kPlaneB, g.n0)[p], plane(c, pr, kPlaneC, g.n0)[p],
             &un, &vn);
  float* du = uv_buf(c, pr, dst_code, g.n0);
  du[p] = un;
  du[n + p] = vn;
}

// ---------------------------------------------------------------------------
// Temporally blocked Jacobi: `ns` sweeps per launch on a register tile.
//
// A workgroup of NW waves owns a tile of 128 columns x NW*R rows: lane l of
// wave w holds columns ox + 2l, ox + 2l + 1 of rows oy + w*R .. + R-1 (u, v
// and the coefficients a, b, c, all in VGPRs).  Horizontal neighbours of the
// two columns come from the adjacent lane through DPP wave shifts folded
// into the adds; vertical neighbours are the thread's own rows, and the rows
// across a wave boundary go through a small double-buffered LDS exchange
// (one barrier per sweep).  The tile carries a halo of `halo` >= ns pixels on
// every side, loaded with mirrored (half-sample symmetric) coordinates:
// reflecting u, v and the coefficients at the image border makes every
// mirrored pixel evolve exactly like its mirror image (the sums are single
// commutative adds), which is the clamp-to-edge neighbourhood of the
// reference iteration, bitwise.  Each sweep invalidates one more ring of the
// halo; after ns sweeps the interior (128 - 2 halo) x (NW*R - 2 halo) pixels
// equal ns sweeps of the one-sweep kernel and are stored.
__device__ __forceinline__ int32_t reflect(int32_t c, int32_t n) {
  c = (c < 0) ? -1 - c : c;
  c = (c >= n) ? 2 * n - 1 - c : c;
  return min(max(c, 0), n - 1);
}
__device__ __forceinline__ float dpp_from_left(float x) {   // lane l receives lane l-1
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float x) {  // lane l receives lane l+1
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
}

template <int R, int NW>
__global__ void __launch_bounds__(64 * NW) k_hs_jacobi_tb(ChunkPtrs c, LevelGeom g, int32_t src_code, int32_t dst_code,
                                                          int32_t ns, int32_t halo, int32_t tiles_x,
                                                          int32_t tiles_per_pair) {
  constexpr int TH = NW * R;
  __shared__ float4 xch[2][NW][2][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t pr = blockIdx.x / tiles_per_pair;
  if (c.active && !c.active[pr]) return;  // uniform over the workgroup, before any barrier
  const int32_t t = blockIdx.x % tiles_per_pair;
  const int32_t ty = t / tiles_x, tx = t % tiles_x;
  const int32_t ox = tx * (128 - 2 * halo) - halo;
  const int32_t oy = ty * (TH - 2 * halo) - halo;
  const int64_t n = (int64_t)g.w * g.h;
  const float* su = uv_buf(c, pr, src_code, g.n0);
  const float* sv = su + n;
  const float* pa = plane(c, pr, kPlaneA, g.n0);
  const float* pb = plane(c, pr, kPlaneB, g.n0);
  const float* pc = plane(c, pr, kPlaneC, g.n0);
  const int32_t cx0 = ox + 2 * lane, cx1 = cx0 + 1;
  const int32_t gx0 = reflect(cx0, g.w), gx1 = reflect(cx1, g.w);

  float u[2][R], v[2][R], A[2][R], B[2][R], C[2][R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = (int64_t)reflect(oy + w * R + r, g.h) * g.w;
    u[0][r] = su[row + gx0];
    u[1][r] = su[row + gx1];
    v[0][r] = sv[row + gx0];
    v[1][r] = sv[row + gx1];
    A[0][r] = pa[row + gx0];
    A[1][r] = pa[row + gx1];
    B[0][r] = pb[row + gx0];
    B[1][r] = pb[row + gx1];
    C[0][r] = pc[row + gx0];
    C[1][r] = pc[row + gx1];
  }

  for (int s = 0; s < ns; ++s) {
    const int slot = s & 1;
    xch[slot][w][0][lane] = make_float4(u[0][0], u[1][0], v[0][0], v[1][0]);
    xch[slot][w][1][lane] = make_float4(u[0][R - 1], u[1][R - 1], v[0][R - 1], v[1][R - 1]);
    __syncthreads();
    const float4 up = (w > 0) ? xch[slot][w - 1][1][lane] : xch[slot][w][0][lane];
    const float4 dn = (w < NW - 1) ? xch[slot][w + 1][0][lane] : xch[slot][w][1][lane];
    float pu0 = up.x, pu1 = up.y, pv0 = up.z, pv1 = up.w;  // old values of the row above
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float nu0 = (r + 1 < R) ? u[0][r + 1] : dn.x;
      const float nu1 = (r + 1 < R) ? u[1][r + 1] : dn.y;
      const float nv0 = (r + 1 < R) ? v[0][r + 1] : dn.z;
      const float nv1 = (r + 1 < R) ? v[1][r + 1] : dn.w;
      // vertical pair sums and [1 2 1] columns
      const float qu0 = pu0 + nu0, qu1 = pu1 + nu1, qv0 = pv0 + nv0, qv1 = pv1 + nv1;
      const float cu0 = fmaf(u[0][r], 2.f, qu0), cu1 = fmaf(u[1][r], 2.f, qu1);
      const float cv0 = fmaf(v[0][r], 2.f, qv0), cv1 = fmaf(v[1][r], 2.f, qv1);
      // horizontal: column 0's left is the left lane's column 1; column 1's right is the right lane's column 0
      const float ub0 = jac_bar(qu0, dpp_from_left(cu1), cu1);
      const float ub1 = jac_bar(qu1, cu0, dpp_from_right(cu0));
      const float vb0 = jac_bar(qv0, dpp_from_left(cv1), cv1);
      const float vb1 = jac_bar(qv1, cv0, dpp_from_right(cv0));
      pu0 = u[0][r];
      pu1 = u[1][r];
      pv0 = v[0][r];
      pv1 = v[1][r];
      jac_update(ub0, vb0, A[0][r], B[0][r], C[0][r], &u[0][r], &v[0][r]);
      jac_update(ub1, vb1, A[1][r], B[1][r], C[1][r], &u[1][r], &v[1][r]);
    }
  }

  float* du = uv_buf(c, pr, dst_code, g.n0);
  float* dv = du + n;
  const bool in0 = (cx0 >= ox + halo) && (cx0 < ox + 128 - halo) && (cx0 < g.w);
  const bool in1 = (cx1 >= ox + halo) && (cx1 < ox + 128 - halo) && (cx1 < g.w);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int32_t yy = oy + w * R + r;
    if (yy < oy + halo || yy >= oy + TH - halo || yy >= g.h) continue;
    const int64_t row = (int64_t)yy * g.w;
    if (in0) {
      du[row + cx0] = u[0][r];
      dv[row + cx0] = v[0][r];
    }
    if (in1) {
      du[row + cx1] = u[1][r];
      dv[row + cx1] = v[1][r];
    }
  }
}

// ---------------------------------------------------------------------------
// Streaming temporally blocked Jacobi ("2.5-D"): one wave owns a strip of 128
// columns (two per lane, mirrored halo of K columns each side) and a band of
// rows, and streams down it: each step reads one input row (u, v, a, b, c)
// and advances every row in flight by one sweep, so that after the step
// sweep s holds row i - s.  Sweep s keeps its last three rows in VGPRs (the
// step loop is unrolled by 3 so their slots are static); the coefficients of
// the last K input rows sit in a per-wave LDS ring.  There is no vertical
// halo tile and no barrier: waves are independent, which lets the loads of
// one wave overlap the arithmetic of another.  Rows above and below the
// image are mirrored, which reproduces clamp-to-edge bitwise (same argument
// as for the tile kernel).  Exactly K sweeps run per launch: with a run-time
// count the window slots become run-time selections (about one extra move
// per arithmetic instruction), so shorter passes use a smaller K instance.
// One input step of the streaming kernel: input row ii enters sweep 0 and
// every sweep s <= K advances row ii - s.  U = ii mod 3 and the sweep index
// are template parameters so that every window slot is a compile-time
// register (template recursion instead of a loop the compiler may not unroll).
// Per-lane element at a wave-uniform base: the address is base + a 32-bit
// lane offset.  The pointers are global-memory pointers (address space 1):
// generic (flat) accesses would also count against the LDS wait counter, so
// every wait for the LDS ring would also wait for the rows in flight.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) const float gcfloat;
__device__ __forceinline__ gcfloat& at_off(const float* base, uint32_t byte_off) {
  asm("" : "+v"(byte_off));
  return *(gcfloat*)((gcchar*)base + byte_off);
}
__device__ __forceinline__ gfloat& at_off(float* base, uint32_t byte_off) {
  asm("" : "+v"(byte_off));
  return *(gfloat*)((gchar*)base + byte_off);
}

// Row bands per pair of a streaming Jacobi launch over `n` pairs without a
// tuned choice: enough waves (`want`) to fill the chip, but no band shorter
// than 64 rows (each band re-reads a 2K + 3 row halo) or taller than `cap`.
inline int32_t stream_bands(int32_t h, int32_t strips, int64_t n, int32_t want, int32_t cap) {
  int64_t bh = (int64_t)h * strips * (n > 1 ? n : 1) / want;
  bh = bh < 64 ? 64 : (bh > cap ? cap : bh);
  return (int32_t)((h + bh - 1) / bh);
}

// Row bands per pair for a walk over a device-built list of `n` pairs by
// `slots` resident waves: the band count (bands of 4 rows up to `cap`) that
// minimises rounds of waves x rows a wave streams (band + halo); a wave's
// rows run one after another, so short bands help when few pairs are
// listed, and fewer, taller bands re-read less halo when many are.
// (A heuristic: evaluated in FP32, once per wave.)
__device__ inline int32_t list_bands(int32_t h, int32_t strips, int64_t n, int32_t slots, int32_t cap, int32_t halo) {
  const float per_band = (float)strips * (float)(n > 1 ? n : 1) / (float)slots;  // rounds per band of each pair
  int32_t best = (h + cap - 1) / cap;
  float best_cost = 3.0e38f;
  const int32_t b_max = max(best, min(h / 4, 32));
  for (int32_t b = best; b <= b_max; ++b) {
    const int32_t bh = (h + b - 1) / b;
    const float cost = ceilf(per_band * (float)b) * (float)(bh + halo);
    if (cost < best_cost) {
      best_cost = cost;
      best = b;
    }
  }
  return best;
}

template <int K>
struct StStep {
  float4 (&win)[K][3];
  float2 (&ring)[K][3][64];
  int lane;
  int32_t y0, y1, w;
  float* du;
  float* dv;
  uint32_t bo0, bo1;  // byte offsets of the lane's two output columns
  bool in0, in1;
  bool vec;           // wave-uniform: 8-byte accesses (see the kernel)

  struct Coef {
    float2 a, b, c;
  };
  __device__ __forceinline__ Coef ring_row(int32_t row) const {
    const int rr = ((row % K) + K) % K;
    return Coef{ring[rr][0][lane], ring[rr][1][lane], ring[rr][2][lane]};
  }

  // Sweep S advances row ii - S with the coefficients `co` of that row,
  // which were read from the ring one sweep earlier (the reads of sweep
  // S + 1's row are issued ahead of sweep S's arithmetic); `last` holds row
  // ii - K for sweep K, read at the start of the step.
  template <int U, int S>
  __device__ __forceinline__ void sweep(int32_t ii, const Coef& co, const Coef& last) {
    if constexpr (S <= K) {
      Coef nx;
      if constexpr (S + 1 < K) {
        nx = ring_row(ii - S - 1);
        __builtin_amdgcn_sched_barrier(0);
      } else if constexpr (S + 1 == K) {
        nx = last;
      }
      const float4 A = win[S - 1][(U - S + 2 + 3 * K) % 3];
      const float4 B = win[S - 1][(U - S + 3 * K) % 3];
      const float4 C = win[S - 1][(U - S + 1 + 3 * K) % 3];
      const float2 ca = co.a, cb = co.b, cc = co.c;
      const float qu0 = A.x + C.x, qu1 = A.y + C.y, qv0 = A.z + C.z, qv1 = A.w + C.w;
      const float cu0 = fmaf(B.x, 2.f, qu0), cu1 = fmaf(B.y, 2.f, qu1);
      const float cv0 = fmaf(B.z, 2.f, qv0), cv1 = fmaf(B.w, 2.f, qv1);
      const float ub0 = jac_bar(qu0, dpp_from_left(cu1), cu1);
      const float ub1 = jac_bar(qu1, cu0, dpp_from_right(cu0));
      const float vb0 = jac_bar(qv0, dpp_from_left(cv1), cv1);
      const float vb1 = jac_bar(qv1, cv0, dpp_from_right(cv0));
      float4 N;
      jac_update(ub0, vb0, ca.x, cb.x, cc.x, &N.x, &N.z);
      jac_update(ub1, vb1, ca.y, cb.y, cc.y, &N.y, &N.w);
      if constexpr (S < K) win[S][(U - S + 3 * K) % 3] = N;
      if constexpr (S == K) {
        // keep the last sweep's arithmetic ahead of the lane-masked stores
        // (sunk into them, its wave shifts could not fold into the adds)
        asm volatile("" ::"v"(N.x), "v"(N.y), "v"(N.z), "v"(N.w));
        const int32_t r = ii - S;
        if (r >= y0 && r < y1) {
          float* ru = du + (int64_t)r * w;
          float* rv = dv + (int64_t)r * w;
          if (vec) {
            // adjacent, 8-byte aligned columns, and in0 == in1 (K, the strip
            // origin and the width are even on this path): one 8-byte store
            typedef float nf2 __attribute__((ext_vector_type(2)));
            typedef __attribute__((address_space(1))) nf2 gnf2;
            if (in0) {
              *(gnf2*)&at_off(ru, bo0) = nf2{N.x, N.y};
              *(gnf2*)&at_off(rv, bo0) = nf2{N.z, N.w};
            }
          } else {
            if (in0) {
              at_off(ru, bo0) = N.x;
              at_off(rv, bo0) = N.z;
            }
            if (in1) {
              at_off(ru, bo1) = N.y;
              at_off(rv, bo1) = N.w;
            }
          }
        }
        return;
      }
      sweep<U, S + 1>(ii, nx, last);
    }
  }

  // Input row ii sits in prefetch slot U of P (P a multiple of 3, so that
  // ii mod 3 = U mod 3 selects the window slot); once it has entered the
  // window and the ring, the slot is refilled with row ii + P (P rows of
  // loads in flight per wave).  The ring has K slots: row ii takes the slot
  // of row ii - K, whose coefficients (needed by sweep K in this step) are
  // read first; the LDS operations of a wave execute in order.
  template <int U, int P, typename F>
  __device__ __forceinline__ void step(int32_t ii, float4 (&nuv)[P], float2 (&na)[P], float2 (&nb)[P],
                                       float2 (&nc)[P], F&& load_row) {
    constexpr int W = U % 3;
    win[0][W] = nuv[U];
    const Coef last = ring_row(ii - K);
    const int rs = ((ii % K) + K) % K;
    ring[rs][0][lane] = na[U];
    ring[rs][1][lane] = nb[U];
    ring[rs][2][lane] = nc[U];
    load_row(ii + P, nuv[U], na[U], nb[U], nc[U]);
    if constexpr (K == 1) sweep<W, 1>(ii, last, last);
    else sweep<W, 1>(ii, ring_row(ii - 1), last);
  }
  // steps U .. P-1 of one loop iteration (rows i + U ..)
  template <int U, int P, typename F>
  __device__ __forceinline__ void steps(int32_t i, float4 (&nuv)[P], float2 (&na)[P], float2 (&nb)[P],
                                        float2 (&nc)[P], F&& load_row) {
    step<U, P>(i + U, nuv, na, nb, nc, load_row);
    if constexpr (U + 1 < P) steps<U + 1, P>(i, nuv, na, nb, nc, load_row);
  }
};

template <int K, int P, int WB>
__global__ void __launch_bounds__(64 * WB) k_hs_jacobi_st(ChunkPtrs c, LevelGeom g, int32_t src_code, int32_t dst_code,
                                                      int32_t strips, int32_t bands, int32_t band_h, int32_t slots,
                                                      int32_t band_cap) {
  __shared__ float2 ring[WB][K][3][64];  // [wave][row slot][a, b, c][lane] (two columns per lane)
  const int lane = threadIdx.x & 63;
  // wave-uniform from here on: the pair, band, strip, row counters and plane
  // pointers live in SGPRs and their arithmetic runs on the scalar unit
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // With an active-pair list the number of listed pairs is known here only:
  // the bands are chosen from it (list_bands; `slots` = the grid's waves).
  int64_t listed = 0;
  if (c.act_list) {
    listed = *c.act_count;
    if (listed == 0) return;
    bands = list_bands(g.h, strips, listed, slots, band_cap, 2 * K + 3);
    band_h = (g.h + bands - 1) / bands;
  }
  const int64_t per_pair = (int64_t)strips * bands;
  // A wave takes unit (pair, band, strip) = its index; with an active-pair
  // list the units index list slots, and the resident grid strides over them
  // until the list is exhausted.
  for (int64_t unit = (int64_t)xcd_block(blockIdx.x, gridDim.x) * WB + wv;; unit += (int64_t)gridDim.x * WB) {
    int64_t pr;
    if (c.act_list) {
      const int64_t slot = unit / per_pair;
      if (slot >= listed) return;
      pr = c.act_list[slot];
    } else {
      pr = unit / per_pair;
      if (pr >= c.n_pairs) return;
      if (c.active && !c.active[pr]) return;
    }
    const int32_t rem = (int32_t)(unit % per_pair);
    const int32_t band = rem / strips, strip = rem % strips;
    const int32_t ox = strip * (128 - 2 * K) - K;
    const int32_t y0 = band * band_h, y1 = min(g.h, y0 + band_h);
    const int64_t n = (int64_t)g.w * g.h;
    const float* su = uv_buf(c, pr, src_code, g.n0);
    const float* sv = su + n;
    const float* pa = plane(c, pr, kPlaneA, g.n0);
    const float* pb = plane(c, pr, kPlaneB, g.n0);
    const float* pc = plane(c, pr, kPlaneC, g.n0);
    float* du = uv_buf(c, pr, dst_code, g.n0);
    float* dv = du + n;
    const int32_t cx0 = ox + 2 * lane, cx1 = cx0 + 1;
    const int32_t gx0 = reflect(cx0, g.w), gx1 = reflect(cx1, g.w);
    const bool in0 = (cx0 >= ox + K) && (cx0 < ox + 128 - K) && (cx0 < g.w);
    const bool in1 = (cx1 >= ox + K) && (cx1 < ox + 128 - K) && (cx1 < g.w);

    // sweep windows: win[s][slot] = (u col0, u col1, v col0, v col1) of sweep s's row with row % 3 == slot
    float4 win[K][3];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
      for (int q = 0; q < 3; ++q) win[s][q] = make_float4(0.f, 0.f, 0.f, 0.f);

    int32_t i = y0 - K - 1;
    i -= ((i % 3) + 3) % 3;  // start on a multiple of 3 so that slots are static
    const int32_t i_end = y1 - 1 + K;
    // Rows are read as float2 where a lane's two columns are adjacent and the
    // pair is 8-byte aligned in every row (even width, even first column);
    // lanes whose columns are mirrored at the image border read scalars.
    // The float2 path is taken by whole waves (interior strips); a wave with
    // a mirrored border column reads scalars.
    const bool lane_vec = (g.w % 2 == 0) && (K % 2 == 0) && (gx1 == gx0 + 1) && (gx0 % 2 == 0) &&
                          ((reinterpret_cast<uintptr_t>(su) | reinterpret_cast<uintptr_t>(sv) |
                            reinterpret_cast<uintptr_t>(pa) | reinterpret_cast<uintptr_t>(pb) |
                            reinterpret_cast<uintptr_t>(pc) | reinterpret_cast<uintptr_t>(du) |
                            reinterpret_cast<uintptr_t>(dv)) % 8 == 0);
    const bool vec = __all(lane_vec);
    const uint32_t bo0 = 4u * (uint32_t)gx0, bo1 = 4u * (uint32_t)gx1;
    auto load_row = [&](int32_t row, float4& uv, float2& a, float2& b, float2& cc) {
      const int64_t r = (int64_t)reflect(row, g.h) * g.w;
      const float *ru = su + r, *rv = sv + r, *ra = pa + r, *rb = pb + r, *rc = pc + r;
      if (vec) {
        typedef float nf2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) const nf2 gcnf2;
        const nf2 u2 = *(gcnf2*)&at_off(ru, bo0);
        const nf2 v2 = *(gcnf2*)&at_off(rv, bo0);
        const nf2 a2 = *(gcnf2*)&at_off(ra, bo0);
        const nf2 b2 = *(gcnf2*)&at_off(rb, bo0);
        const nf2 c2 = *(gcnf2*)&at_off(rc, bo0);
        uv = make_float4(u2.x, u2.y, v2.x, v2.y);
        a = make_float2(a2.x, a2.y);
        b = make_float2(b2.x, b2.y);
        cc = make_float2(c2.x, c2.y);
      } else {
        uv = make_float4(at_off(ru, bo0), at_off(ru, bo1), at_off(rv, bo0), at_off(rv, bo1));
        a = make_float2(at_off(ra, bo0), at_off(ra, bo1));
        b = make_float2(at_off(rb, bo0), at_off(rb, bo1));
        cc = make_float2(at_off(rc, bo0), at_off(rc, bo1));
      }
    };
    float4 nuv[P];
    float2 na[P], nb[P], nc[P];
#pragma unroll
    for (int q = 0; q < P; ++q) load_row(i + q, nuv[q], na[q], nb[q], nc[q]);
    StStep<K> st{win, ring[wv], lane, y0, y1, g.w, du, dv, 4u * (uint32_t)cx0, 4u * (uint32_t)cx1, in0, in1, vec};
    static_assert(P % 3 == 0, "prefetch depth must be a multiple of the 3 window slots");
    for (; i <= i_end; i += P) st.template steps<0, P>(i, nuv, na, nb, nc, load_row);
    if (!c.act_list) return;  // one unit per wave without a list
  }
}

// Warm-start schedule: the pairs at position `step` of their work packet
// (flags, the ordered list of their chunk slots and its length), and for
// the cold step the frames whose pyramids those pairs need.  One workgroup;
// chunks hold at most a few thousand pairs.
__global__ void __launch_bounds__(256) k_warm_step(const PairDesc* __restrict__ pairs, int64_t n_pairs, int32_t step,
                                                   uint8_t* __restrict__ active, uint8_t* __restrict__ factive,
                                                   int64_t n_frames, int32_t* __restrict__ list,
                                                   int32_t* __restrict__ count) {
  __shared__ int32_t part[256];
  const int t = threadIdx.x;
  if (factive)
    for (int64_t f = t; f < n_frames; f += 256) factive[f] = 0;
  __syncthreads();
  const int64_t per = (n_pairs + 255) / 256, b0 = min(n_pairs, (int64_t)t * per), b1 = min(n_pairs, b0 + per);
  int32_t cnt = 0;
  for (int64_t i = b0; i < b1; ++i) {
    const bool a = pairs[i].pos == step;
    active[i] = a ? 1 : 0;
    cnt += a ? 1 : 0;
    if (a && factive) {  // racing stores of the same value
      factive[pairs[i].f1] = 1;
      factive[pairs[i].f2] = 1;
    }
  }
  part[t] = cnt;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan
    const int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t at = part[t] - cnt;
  for (int64_t i = b0; i < b1; ++i)
    if (pairs[i].pos == step) list[at++] = (int32_t)i;
  if (t == 255) *count = part[255];
}

LevelGeom level_geom(const FlowGroup& grp, int32_t l) {
  LevelGeom g;
  g.w = grp.dims[l].w;
  g.h = grp.dims[l].h;
  g.has_coarse = (l + 1 < (int32_t)grp.dims.size()) ? 1 : 0;
  g.cw = g.has_coarse ? grp.dims[l + 1].w : 0;
  g.ch = g.has_coarse ? grp.dims[l + 1].h : 0;
  g.n0 = (int64_t)grp.w * grp.h;
  g.lvl_off = (int64_t)grp.lvl_off[l];
  g.level = l;
  return g;
}

}  // namespace

// Jacobi kernel variants: (rows per wave, waves per workgroup); variant 0 is
// the one-sweep reference kernel.  Streaming variants use rows = 0, waves =
// the largest sweep count K, cap their band height at band_cap rows (taller
// bands re-read fewer halo rows but give fewer waves) and keep `prefetch`
// input rows in flight per wave (3 or, for K = 10 passes, 6; 9 was measured
// no faster than 6).
struct JacobiVariant {
  int32_t rows, waves, band_cap, prefetch;
};
constexpr JacobiVariant kVariants[] = {{1, 4, 0, 0},     {8, 16, 0, 0},    {16, 8, 0, 0},    {8, 8, 0, 0},
                                       {4, 16, 0, 0},    {0, 6, 256, 3},   {0, 8, 256, 3},   {0, 10, 256, 3},
                                       {0, 10, 1024, 3}, {0, 10, 256, 6},  {0, 10, 1024, 6}, {0, 12, 256, 3},
                                       {0, 12, 1024, 3}, {0, 12, 256, 6},  {0, 12, 1024, 6}, {0, 13, 256, 3},
                                       {0, 13, 1024, 3}, {0, 17, 256, 3},  {0, 17, 1024, 3}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kDefaultStreaming = 9;  // K <= 10, 6 rows in flight: the masked (fallback) default

struct JacobiChoice {
  int32_t variant;    // index into kVariants
  int32_t k;          // sweeps per pass (= halo)
  int32_t bands = 0;  // streaming variants: row bands per pair (0: sized from the pair count)
};

// Compute units of the current device (queried once per device).
static int device_cus() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    cached[dev] = (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) ? n : 256;
  }
  return cached[dev];
}

bool variant_fits(int v, int32_t k, const LevelGeom& g) {
  if (v == 0) return k == 1;
  if (kVariants[v].rows == 0) return k >= 1 && k <= kVariants[v].waves && kVariants[v].waves <= g.w &&
                                     kVariants[v].waves + 4 <= g.h;
  const int32_t th = kVariants[v].rows * kVariants[v].waves;
  return k >= 1 && 2 * k < 128 && 2 * k < th && k <= g.w && k <= g.h;
}

scn_status launch_jacobi(const JacobiChoice& jc, const ChunkPtrs& c, const LevelGeom& g, int64_t n_pairs,
                         int32_t src, int32_t dst, int32_t ns, hipStream_t s) {
  static constexpr const char* kLevelTimer[] = {"hs_jacobi_l0", "hs_jacobi_l1", "hs_jacobi_l2", "hs_jacobi_l3",
                                                "hs_jacobi_l4", "hs_jacobi_l5", "hs_jacobi_l6"};
  // work units: pixels of the level x pairs per pass over the planes (each
  // launch of the one-sweep kernel is a pass; 0 for a masked pass, whose pair
  // count is known only on the device)
  const double units = c.active ? 0.0 : (double)g.w * g.h * (double)n_pairs * (jc.variant == 0 ? ns : 1);
  KernelTimer timer("hs_jacobi", s, units);
  KernelTimer timer_l(kLevelTimer[std::min(g.level, 6)], s, units);
  if (jc.variant == 0) {
    const int64_t bpp = ((int64_t)g.w * g.h + kThreads - 1) / kThreads;
    for (int32_t it = 0; it < ns; ++it) {
      const int32_t d = (it == ns - 1) ? dst : (it % 2 == 0 ? 1 - src : src);
      const int32_t sc = (it == 0) ? src : (it % 2 == 1 ? 1 - src : src);
      hipLaunchKernelGGL(k_hs_jacobi1, dim3((unsigned)(bpp * n_pairs)), dim3(kThreads), 0, s, c, g, sc, d,
                         (int32_t)bpp);
    }
    SCN_LAUNCHED("jacobi launch");
    return SCN_OK;
  }
  const JacobiVariant v = kVariants[jc.variant];
  if (v.rows == 0) {
    // the streaming kernel runs exactly K sweeps (a compile-time count: the
    // window registers then need no run-time selection); a pass of ns <= the
    // variant's maximum uses the K = ns instance
    const int32_t K = ns;
    if (K < 1 || K > v.waves) { set_error("internal: bad streaming Jacobi sweep count"); return SCN_EINVAL; }
    const int32_t strips = (g.w + (128 - 2 * K) - 1) / (128 - 2 * K);
    // bands: enough independent waves to fill the chip (about 24 per CU).
    // With an active mask but no list (not used by the library's own paths)
    // the active count is unknown here: bands sized for one pair in eight.
    // With a list the kernel chooses the bands from the listed count itself.
    const int64_t n_eff = c.active ? std::max<int64_t>(1, (n_pairs + 7) / 8) : n_pairs;
    int32_t bands = stream_bands(g.h, strips, n_eff, 24 * device_cus(), v.band_cap);
    // a tuned band count (the tail of the last round of waves depends on it)
    if (jc.bands > 0 && !c.active) {
      const int32_t b = std::min(jc.bands, g.h), bh = (g.h + b - 1) / b;
      bands = (g.h + bh - 1) / bh;
    }
    const int32_t band_h = (g.h + bands - 1) / bands;
    const int64_t units = (int64_t)strips * bands * n_pairs;
    // Waves per workgroup: each wave's coefficient ring takes K x 1.5 KiB of
    // LDS, so that 8 waves (two workgroups) fit a CU's 160 KiB up to K = 13;
    // larger K run one wave per workgroup (6 or 7 per CU).
    const int wb = K <= 13 ? 4 : 1;
    int64_t grid = (units + wb - 1) / wb;
    // a list walk runs on a resident grid (8 waves per CU): the waves stride
    // over the listed pairs' units, and an empty list costs one short launch
    if (c.act_list) grid = (int64_t)device_cus() * (8 / wb);
    const int32_t slots = c.act_list ? (int32_t)(grid * wb) : 0;
    if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
    const dim3 gd((unsigned)grid), bd(64 * wb);
    if (K == 10 && v.prefetch == 6) {
      hipLaunchKernelGGL((k_hs_jacobi_st<10, 6, 4>), gd, bd, 0, s, c, g, src, dst, strips, bands, band_h, slots,
                         v.band_cap);
    } else if (K == 12 && v.prefetch == 6) {
      hipLaunchKernelGGL((k_hs_jacobi_st<12, 6, 4>), gd, bd, 0, s, c, g, src, dst, strips, bands, band_h, slots,
                         v.band_cap);
    } else {
      switch (K) {
#define SCN_ST(k, wbk) \
  case k:                                                                                                     \
    hipLaunchKernelGGL((k_hs_jacobi_st<k, 3, wbk>), gd, bd, 0, s, c, g, src, dst, strips, bands, band_h, slots, \
                       v.band_cap);                                                                              \
    break;
        SCN_ST(1, 4) SCN_ST(2, 4) SCN_ST(3, 4) SCN_ST(4, 4) SCN_ST(5, 4) SCN_ST(6, 4) SCN_ST(7, 4) SCN_ST(8, 4)
        SCN_ST(9, 4) SCN_ST(10, 4) SCN_ST(11, 4) SCN_ST(12, 4) SCN_ST(13, 4) SCN_ST(14, 1) SCN_ST(15, 1)
        SCN_ST(16, 1) SCN_ST(17, 1)
#undef SCN_ST
        default: set_error("internal: bad streaming Jacobi sweep count"); return SCN_EINVAL;
      }
    }
    SCN_LAUNCHED("jacobi launch");
    return SCN_OK;
  }
  const int32_t th = v.rows * v.waves;
  const int32_t tiles_x = (g.w + (128 - 2 * jc.k) - 1) / (128 - 2 * jc.k);
  const int32_t tiles_y = (g.h + (th - 2 * jc.k) - 1) / (th - 2 * jc.k);
  const int64_t tpp = (int64_t)tiles_x * tiles_y;
  const int64_t grid = tpp * n_pairs;
  if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
  const dim3 gd((unsigned)grid), bd(64 * v.waves);
  switch (jc.variant) {
    case 1: hipLaunchKernelGGL((k_hs_jacobi_tb<8, 16>), gd, bd, 0, s, c, g, src, dst, ns, jc.k, tiles_x, (int32_t)tpp); break;
    case 2: hipLaunchKernelGGL((k_hs_jacobi_tb<16, 8>), gd, bd, 0, s, c, g, src, dst, ns, jc.k, tiles_x, (int32_t)tpp); break;
    case 3: hipLaunchKernelGGL((k_hs_jacobi_tb<8, 8>), gd, bd, 0, s, c, g, src, dst, ns, jc.k, tiles_x, (int32_t)tpp); break;
    case 4: hipLaunchKernelGGL((k_hs_jacobi_tb<4, 16>), gd, bd, 0, s, c, g, src, dst, ns, jc.k, tiles_x, (int32_t)tpp); break;
    default: set_error("internal: bad Jacobi variant"); return SCN_EINVAL;
  }
  SCN_LAUNCHED("jacobi launch");
  return SCN_OK;
}

// Default schedule without tuning: 10 sweeps per pass on 128 x 128 tiles.
JacobiChoice default_choice(const LevelGeom& g, int32_t iters) {
  for (int32_t k : {10, 8, 5, 4, 3, 2})
    if (k <= iters && variant_fits(1, k, g)) return JacobiChoice{1, k};
  return JacobiChoice{0, 1};
}

#include "tune.inc"

namespace {
#include "farneback.inc"
}  // namespace

// Levels 1..L-1 of every frame slot of a chunk.
scn_status launch_pyramids(const ChunkPtrs& c, const FlowGroup& grp, const FlowChunk& ch, int32_t L, hipStream_t s) {
  for (int32_t l = 1; l < L; ++l) {
    const LevelGeom sg = level_geom(grp, l - 1), dg = level_geom(grp, l);
    const int32_t tiles_x = (dg.w + kPyrTW - 1) / kPyrTW, tiles_y = (dg.h + kPyrTH - 1) / kPyrTH;
    const int64_t tpf = (int64_t)tiles_x * tiles_y;
    const int64_t grid = tpf * ch.n_frames;
    if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
    KernelTimer timer("pyr_down", s);
    if (l == 1)
      hipLaunchKernelGGL(k_pyr_down<true>, dim3((unsigned)grid), dim3(256), 0, s, c, sg, dg, tiles_x, (int32_t)tpf);
    else
      hipLaunchKernelGGL(k_pyr_down<false>, dim3((unsigned)grid), dim3(256), 0, s, c, sg, dg, tiles_x, (int32_t)tpf);
    SCN_LAUNCHED("pyramid launch");
  }
  return SCN_OK;
}

// Expansion constants for the Gaussian applicability of standard deviation
// sigma over the 5 x 5 window (double precision, rounded once to float).
FbConst fb_constants(float sigma) {
  double gg[3];
  for (int t = 0; t < 3; ++t) gg[t] = std::exp(-(double)(t * t) / (2.0 * (double)sigma * sigma));
  // 1-D sums of g(t) t^k over t = -2..2
  const double S0 = gg[0] + 2 * gg[1] + 2 * gg[2], S2 = 2 * gg[1] + 8 * gg[2], S4 = 2 * gg[1] + 32 * gg[2];
  // 2-D sums of a(t) = g(tx) g(ty) times the basis products
  const double s0 = S0 * S0, s2 = S2 * S0, s4 = S4 * S0, s22 = S2 * S2;
  // inverse of the coupled block over the basis (1, tx^2, ty^2)
  const double M[3][3] = {{s0, s2, s2}, {s2, s4, s22}, {s2, s22, s4}};
  const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                     M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                     M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  auto inv = [&](int r, int col) {  // (adj M)[r][col] / det = cofactor(col, r) / det
    const int r0 = (col + 1) % 3, r1 = (col + 2) % 3, c0 = (r + 1) % 3, c1 = (r + 2) % 3;
    return (M[r0][c0] * M[r1][c1] - M[r0][c1] * M[r1][c0]) / det;
  };
  FbConst k;
  k.g0 = (float)gg[0];
  k.g1 = (float)gg[1];
  k.g2 = (float)gg[2];
  k.inv_s2 = (float)(1.0 / s2);
  k.half_inv_s22 = (float)(0.5 / s22);
  k.i10 = (float)inv(1, 0);
  k.i11 = (float)inv(1, 1);
  k.i12 = (float)inv(1, 2);
  k.i20 = (float)inv(2, 0);
  k.i21 = (float)inv(2, 1);
  k.i22 = (float)inv(2, 2);
  return k;
}

// Farneback flow of one chunk: pyramids, then per level (coarse to fine) the
// expansion of every frame slot and `iters` displacement passes over every
// pair, the first from the coarser level's flow.
scn_status run_fb_chunk(const FlowPlan& plan, const FlowGroup& grp, const FlowChunk& ch,
                        const scn_flow_params& prm, void* ws, hipStream_t s) {
  uint8_t* base = (uint8_t*)ws;
  const int32_t L = plan.levels;
  scn_status st;
  ChunkPtrs c;
  c.frames = (const FrameDesc*)(base + ch.frames_off);
  c.pairs = (const PairDesc*)(base + ch.pairs_off);
  c.pyr = (float*)(base + plan.scratch_off);
  c.pyr_floats = (int64_t)grp.pyr_floats;
  c.scratch = (float*)(base + plan.scratch_off + chunk_pyr_bytes(grp, ch));
  c.pair_floats = (int64_t)grp.pair_floats;
  c.n_pairs = ch.n_pairs;
  c.n_frames = ch.n_frames;
  c.active = nullptr;
  c.factive = nullptr;
  c.act_list = nullptr;
  c.act_count = nullptr;
  if (prm.iters == 0) {  // zero prior at every level: the flow is zero
    const int64_t per = 2 * (int64_t)grp.w * grp.h, blocks = (per * ch.n_pairs + 255) / 256;
    if (blocks > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
    KernelTimer timer("fb_disp", s);
    hipLaunchKernelGGL(k_fb_zero, dim3((unsigned)blocks), dim3(256), 0, s, c, per);
    SCN_LAUNCHED("zero flow launch");
    return SCN_OK;
  }
  if ((st = launch_pyramids(c, grp, ch, L, s)) != SCN_OK) return st;
  const FbConst k = fb_constants(prm.fb_sigma);
  const int32_t m = prm.fb_win;
  const FbDisp dp{m, (float)(1.0 / ((2.0 * m + 1) * (2.0 * m + 1))), prm.fb_lambda, (int64_t)grp.exp_off};
  int32_t result = -1;  // buffer code holding the coarser level's flow
  for (int32_t l = L - 1; l >= 0; --l) {
    const LevelGeom g = level_geom(grp, l);
    {
      const int32_t tiles_x = (g.w + kFpTW - 1) / kFpTW, tiles_y = (g.h + kFpTH - 1) / kFpTH;
      const int64_t tpf = (int64_t)tiles_x * tiles_y, grid = tpf * ch.n_frames;
      if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
      KernelTimer timer("fb_poly", s);
      if (l == 0)
        hipLaunchKernelGGL(k_fb_poly<true>, dim3((unsigned)grid), dim3(256), 0, s, c, g, k, dp.exp_off, tiles_x,
                           (int32_t)tpf);
      else
        hipLaunchKernelGGL(k_fb_poly<false>, dim3((unsigned)grid), dim3(256), 0, s, c, g, k, dp.exp_off, tiles_x,
                           (int32_t)tpf);
      SCN_LAUNCHED("expansion launch");
    }
    const int32_t tiles_x = (g.w + kFdTW - 1) / kFdTW, tiles_y = (g.h + kFdTH - 1) / kFdTH;
    const int64_t tpp = (int64_t)tiles_x * tiles_y, grid = tpp * ch.n_pairs;
    if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
    int32_t cur = result;
    for (int32_t it = 0; it < prm.iters; ++it) {
      const int32_t mode = it > 0 ? 2 : (result < 0 ? 0 : 1);
      const int32_t dst = (l == 0 && it == prm.iters - 1) ? 2 : (cur < 0 ? 0 : 1 - cur);
      KernelTimer timer("fb_disp", s);
      const dim3 gd((unsigned)grid), bd(kFdThreads);
      const int32_t src = mode == 0 ? 0 : cur;
      switch (mode * 16 + m) {
#define SCN_FD(md, mm) \
  case md * 16 + mm: hipLaunchKernelGGL((k_fb_disp<md, mm>), gd, bd, 0, s, c, g, dp, src, dst, tiles_x, (int32_t)tpp); break;
#define SCN_FD_M(md) SCN_FD(md, 0) SCN_FD(md, 1) SCN_FD(md, 2) SCN_FD(md, 3) SCN_FD(md, 4) SCN_FD(md, 5) \
  SCN_FD(md, 6) SCN_FD(md, 7) SCN_FD(md, 8)
        SCN_FD_M(0) SCN_FD_M(1) SCN_FD_M(2)
#undef SCN_FD_M
#undef SCN_FD
        default: set_error("internal: bad Farneback box size"); return SCN_EINVAL;
      }
      SCN_LAUNCHED("displacement launch");
      cur = dst;
    }
    result = cur;
  }
  return SCN_OK;
}

// Flow of one chunk of pairs (pyramids, then coarse-to-fine warp, coef and
// Jacobi).  `active` / `factive` (device, per pair / per frame slot) restrict
// the work to a subset of the chunk's pairs (NULL: all).
// One chunk: pyramids, then per level (coarse to fine) setup and Jacobi.  With
// `warm`, the active pairs are solved at level 0 only, from their
// predecessors' flows (PairDesc::init), with prm.iters iterations.
scn_status run_flow_chunk(const FlowPlan& plan, const FlowGroup& grp, const FlowChunk& ch,
                          const scn_flow_params& prm, void* ws, const uint8_t* active, const uint8_t* factive,
                          const int32_t* act_list, const int32_t* act_count, hipStream_t s, bool warm) {
  uint8_t* base = (uint8_t*)ws;
  const float alpha2 = prm.alpha * prm.alpha;
  const int32_t L = plan.levels;
  scn_status st;
  ChunkPtrs c;
  c.frames = (const FrameDesc*)(base + ch.frames_off);
  c.pairs = (const PairDesc*)(base + ch.pairs_off);
  c.pyr = (float*)(base + plan.scratch_off);
  c.pyr_floats = (int64_t)grp.pyr_floats;
  c.scratch = (float*)(base + plan.scratch_off + chunk_pyr_bytes(grp, ch));
  c.pair_floats = (int64_t)grp.pair_floats;
  c.n_pairs = ch.n_pairs;
  c.n_frames = ch.n_frames;
  c.active = active;
  c.factive = factive;
  c.act_list = act_list;
  c.act_count = act_count;
  // pyramids of every frame slot of the chunk (a warm solve reads level 0
  // straight from the table)
  if ((st = launch_pyramids(c, grp, ch, warm ? 1 : L, s)) != SCN_OK) return st;
  int32_t result = -1;  // buffer code holding the coarser level's flow
  for (int32_t l = warm ? 0 : L - 1; l >= 0; --l) {
    const LevelGeom g = level_geom(grp, l);
    const int64_t bpp = ((int64_t)g.w * g.h + kThreads - 1) / kThreads;
    const int64_t grid = bpp * ch.n_pairs;
    if (grid > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
    const int32_t coarse = result < 0 ? 0 : result;
    const int32_t x = result < 0 ? 0 : 1 - result;
    const int32_t start_dst = (l == 0 && prm.iters == 0) ? 2 : x;
    {
      const int32_t tiles_x = (g.w + kSetupTW - 1) / kSetupTW, tiles_y = (g.h + kSetupTH - 1) / kSetupTH;
      const int64_t tpp = (int64_t)tiles_x * tiles_y;
      if (tpp * ch.n_pairs > 0x7FFFFFFF) { set_error("flow chunk too large"); return SCN_EUNSUPPORTED; }
      KernelTimer timer("hs_setup", s);
      // with an active-pair list the grid is resident (four workgroups per
      // CU, fewer if the chunk has fewer tiles) and the workgroups stride over
      // the listed pairs' tiles (as the streaming Jacobi does)
      const int64_t blocks =
          c.act_list ? std::min<int64_t>(tpp * ch.n_pairs, 4LL * device_cus()) : tpp * ch.n_pairs;
      const dim3 grid((unsigned)blocks);
      const bool u8 = g.level == 0, co = g.has_coarse != 0;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, c, g, coarse, start_dst, alpha2, tiles_x, (int32_t)tpp);
      };
      if (c.act_list) {
        if (warm) go(k_hs_setup<true, false, true, true>);
        else if (u8 && co) go(k_hs_setup<true, true, false, true>);
        else if (u8) go(k_hs_setup<true, false, false, true>);
        else if (co) go(k_hs_setup<false, true, false, true>);
        else go(k_hs_setup<false, false, false, true>);
      } else {
        if (warm) go(k_hs_setup<true, false, true, false>);
        else if (u8 && co) go(k_hs_setup<true, true, false, false>);
        else if (u8) go(k_hs_setup<true, false, false, false>);
        else if (co) go(k_hs_setup<false, true, false, false>);
        else go(k_hs_setup<false, false, false, false>);
      }
    }
    SCN_LAUNCHED("setup launch");
    int32_t cur = start_dst;
    if (prm.iters > 0) {
      const JacobiChoice jc = choose_jacobi(grp, l, ch.n_pairs, prm, c, g, cur, s);
      // ceil(iters / k) passes of nearly equal sweep counts (50 = 13+13+12+12
      // rather than 13+13+13+11; results do not depend on the split)
      const int32_t passes = (prm.iters + jc.k - 1) / jc.k;
      for (int32_t done = 0, pass = 0; done < prm.iters; ++pass) {
        const int32_t ns = prm.iters / passes + (pass < prm.iters % passes ? 1 : 0);
        const int32_t dst = (l == 0 && done + ns == prm.iters) ? 2 : 1 - cur;
        st = launch_jacobi(jc, c, g, ch.n_pairs, cur, dst, ns, s);
        if (st != SCN_OK) return st;
        cur = dst;
        done += ns;
      }
    }
    result = cur;
  }
  return SCN_OK;
}

scn_status run_flow(const FlowPlan& plan, const scn_flow_params& prm, void* ws, hipStream_t s) {
  scn_status st = upload_plan(ws, plan.plan_bytes.data(), plan.plan_bytes.size(), s);
  if (st != SCN_OK) return st;
  const bool warm = prm.warm_packet >= 2;
  uint8_t* base = (uint8_t*)ws;
  for (const FlowGroup& grp : plan.groups)
    for (const FlowChunk& ch : grp.chunks) {
      if (plan.solver == SCN_SOLVER_FARNEBACK) {
        if ((st = run_fb_chunk(plan, grp, ch, prm, ws, s)) != SCN_OK) return st;
        continue;
      }
      if (!warm) {
        if ((st = run_flow_chunk(plan, grp, ch, prm, ws, nullptr, nullptr, nullptr, nullptr, s, false)) != SCN_OK)
          return st;
        continue;
      }
      // Warm start: step 0 solves the packets' first pairs cold (masked),
      // step k the pairs at position k from their predecessors' results.  A
      // predecessor lies in this chunk at step k - 1 or in an earlier chunk,
      // so stream order is the dependency order.
      uint8_t* extra = base + plan.scratch_off + chunk_pyr_bytes(grp, ch) + chunk_pairs_bytes(grp, ch);
      uint8_t* active = extra;
      uint8_t* factive = active + align_up((size_t)ch.n_pairs);
      int32_t* list = (int32_t*)(factive + align_up((size_t)ch.n_frames));
      int32_t* count = list + align_up((size_t)ch.n_pairs * 4) / 4;
      const PairDesc* pairs = (const PairDesc*)(base + ch.pairs_off);
      const int32_t steps = ch.max_pos + 1;
      scn_flow_params wp = prm;
      wp.iters = prm.warm_iters;
      for (int32_t k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(k_warm_step, dim3(1), dim3(256), 0, s, pairs, ch.n_pairs, k, active,
                           k == 0 ? factive : nullptr, ch.n_frames, list, count);
        SCN_LAUNCHED("warm step marking launch");
        st = k == 0 ? run_flow_chunk(plan, grp, ch, prm, ws, active, factive, list, count, s, false)
                    : run_flow_chunk(plan, grp, ch, wp, ws, active, nullptr, list, count, s, true);
        if (st != SCN_OK) return st;
      }
    }
  return SCN_OK;
}

}  // namespace scn
