// Sampled-row gather + NV12 -> RGB BT.601 conversion (+ bilinear resize) and
// the fused 16-bin-per-channel HIST, for gfx950.
//
// Conversion (decoder post-processing applied only to sampled rows, Sec. 4.3
// of the Scanner paper; Resize map of Sec. 3.1): BT.601 limited range in Q14
// fixed point,
//   R = clamp((19077 (Y-16) + 26149 (V-128) + 8192) >> 14, 0, 255)
//   G = clamp((19077 (Y-16) -  6419 (U-128) - 13320 (V-128) + 8192) >> 14, 0, 255)
//   B = clamp((19077 (Y-16) + 33050 (U-128) + 8192) >> 14, 0, 255)
// (coefficients = the real BT.601 ones times 2^14, rounded half to even),
// chroma sample (x>>1, y>>1) replicated over its 2x2 block.
//
// HIST (Sec. 5.1.2): bin = channel >> 4.  Since the Q14 sum s decides the
// channel value, bin = clamp(floor(s / 2^18), 0, 15).  The kernel never
// materialises the channel: it forms t = 64 (s + 18 * 2^18) with one 24-bit
// multiply-add per pixel and channel (t is in [0, 2^31) for every input),
// so the top byte of t is floor(s / 2^18) + 18, a "sub-bin" in [0, 52).
// One byte permute turns it into an LDS address (sub-bin * 256 + lane * 4);
// counters are private per lane index (shared by the waves of a workgroup,
// so concurrent waves only meet in the LDS atomic unit), and the clamp to
// [0, 15] is applied once per workgroup when the sub-bins are folded.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace scn {

namespace {

constexpr int kThreads = 256;
constexpr int kSub = 52;           // sub-bins per channel (bins -18 .. 33)
constexpr int kSubBias = 18;
constexpr int kChanBytes = kSub * 256;  // one channel's [sub][lane] table in bytes

// Q14 coefficients.
constexpr int cY = 19077, cRV = 26149, cGU = 6419, cGV = 13320, cBU = 33050;

// Scaled per-block constants: t_c = 64 * (s_c + 18 * 2^18) = kTY * Y + K_c(U, V).
constexpr int kTY = 64 * cY;  // 1220928 < 2^23
constexpr int kBias = kSubBias << 18;
constexpr int kR0 = 64 * (-cRV * 128 + 8192 - 16 * cY + kBias);
constexpr int kG0 = 64 * (cGU * 128 + cGV * 128 + 8192 - 16 * cY + kBias);
constexpr int kB0 = 64 * (-cBU * 128 + 8192 - 16 * cY + kBias);

__device__ __forceinline__ int64_t row_of(const int64_t* rows, int64_t m) { return rows[m]; }

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xFFu; }

// LDS byte address (sub-bin << 8) | lane4 from the top byte of t.
__device__ __forceinline__ uint32_t sub_addr(int t, uint32_t lane4) {
  return __builtin_amdgcn_perm((uint32_t)t, lane4, 0x0C0C0700u);
}

struct BlockK {
  int r, g, b;
};

__device__ __forceinline__ BlockK block_consts(uint32_t u, uint32_t v) {
  BlockK k;
  k.r = (int)v * (64 * cRV) + kR0;
  k.g = (int)u * (-64 * cGU) + ((int)v * (-64 * cGV) + kG0);
  k.b = (int)u * (64 * cBU) + kB0;
  return k;
}

__device__ __forceinline__ void count_px(unsigned char* lds, uint32_t y, const BlockK& k, uint32_t lane4) {
  const int ty = (int)y * kTY;
  const uint32_t ar = sub_addr(ty + k.r, lane4);
  const uint32_t ag = sub_addr(ty + k.g, lane4);
  const uint32_t ab = sub_addr(ty + k.b, lane4);
  atomicAdd(reinterpret_cast<uint32_t*>(lds + ar), 1u);
  atomicAdd(reinterpret_cast<uint32_t*>(lds + kChanBytes + ag), 1u);
  atomicAdd(reinterpret_cast<uint32_t*>(lds + 2 * kChanBytes + ab), 1u);
}

// Two rows of 16 pixels: y0/y1 = 16 luma bytes of each row, uv = 8 (U,V) pairs.
__device__ __forceinline__ void count_seg16(unsigned char* lds, const uint4& y0, const uint4& y1,
                                            const uint4& uv, uint32_t lane4) {
  const uint32_t Y0[4] = {y0.x, y0.y, y0.z, y0.w};
  const uint32_t Y1[4] = {y1.x, y1.y, y1.z, y1.w};
  const uint32_t UV[4] = {uv.x, uv.y, uv.z, uv.w};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // two 2x2 blocks per dword of luma
      const BlockK k = block_consts(byte_of(UV[d], 2 * h), byte_of(UV[d], 2 * h + 1));
      count_px(lds, byte_of(Y0[d], 2 * h), k, lane4);
      count_px(lds, byte_of(Y0[d], 2 * h + 1), k, lane4);
      count_px(lds, byte_of(Y1[d], 2 * h), k, lane4);
      count_px(lds, byte_of(Y1[d], 2 * h + 1), k, lane4);
    }
  }
}

struct FrameGeom {
  const uint8_t* frames;
  int64_t frame_bytes;
  int32_t width, height, pitch;
  int32_t nseg_x;     // full 16-px segments per row pair (vector path), 0 on the scalar path
  int32_t ntail_x;    // remaining 2x2 blocks per row pair
  int32_t chunks;     // workgroups per frame
};

// One workgroup = one chunk of one sampled frame.  Grid: M * chunks.
template <bool kVec>
__global__ void __launch_bounds__(kThreads) k_hist16(FrameGeom g, const int64_t* __restrict__ rows,
                                                     uint32_t* __restrict__ hist) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[3 * kChanBytes];
  __shared__ uint32_t part[3 * kSub];
  const int tid = threadIdx.x;
  const int64_t m = blockIdx.x / g.chunks;
  const int chunk = blockIdx.x % g.chunks;
  for (int i = tid; i < 3 * kChanBytes / 4; i += kThreads) reinterpret_cast<uint32_t*>(lds)[i] = 0u;
  __syncthreads();

  const uint32_t lane4 = (uint32_t)(tid & 63) << 2;
  const uint8_t* frame = g.frames + row_of(rows, m) * g.frame_bytes;
  const uint8_t* uvp = frame + (int64_t)g.pitch * g.height;
  const int32_t rowpairs = g.height >> 1;

  if (kVec) {
    // Segments (16 px x 2 rows) of this chunk, visited with a stride of
    // kThreads; (i, j) advance incrementally instead of dividing each step.
    const int32_t nseg = g.nseg_x * rowpairs;
    const int32_t per = (nseg + g.chunks - 1) / g.chunks;
    const int32_t s0 = chunk * per;
    const int32_t s1 = min(nseg, s0 + per);
    const int32_t di = kThreads % g.nseg_x, dj = kThreads / g.nseg_x;
    int32_t s = s0 + tid;
    int32_t j = s / g.nseg_x, i = s % g.nseg_x;
    // two segments in flight: (a*) is the next one to count, (b*) the one after
    uint4 a0, a1, a2, b0, b1, b2;
    auto load_seg = [&](int32_t jj, int32_t ii, uint4& y0, uint4& y1, uint4& uv) {
      const uint8_t* yr = frame + (int64_t)(2 * jj) * g.pitch + 16 * ii;
      y0 = *reinterpret_cast<const uint4*>(yr);
      y1 = *reinterpret_cast<const uint4*>(yr + g.pitch);
      uv = *reinterpret_cast<const uint4*>(uvp + (int64_t)jj * g.pitch + 16 * ii);
    };
    auto advance = [&]() {
      i += di;
      j += dj;
      if (i >= g.nseg_x) { i -= g.nseg_x; ++j; }
    };
    if (s < s1) load_seg(j, i, a0, a1, a2);
    advance();
    if (s + kThreads < s1) load_seg(j, i, b0, b1, b2);
    for (; s < s1; s += kThreads) {
      const uint4 c0 = a0, c1 = a1, c2 = a2;
      a0 = b0;
      a1 = b1;
      a2 = b2;
      advance();
      if (s + 2 * kThreads < s1) load_seg(j, i, b0, b1, b2);  // two segments ahead
      count_seg16(lds, c0, c1, c2, lane4);
    }
  }
  // 2x2 blocks not covered by 16-px segments (all blocks on the scalar path)
  {
    const int32_t x0 = 16 * g.nseg_x;
    const int64_t nb = (int64_t)g.ntail_x * rowpairs;
    const int64_t per = (nb + g.chunks - 1) / g.chunks;
    const int64_t b0 = (int64_t)chunk * per;
    const int64_t b1 = min(nb, b0 + per);
    for (int64_t b = b0 + tid; b < b1; b += kThreads) {
      const int32_t j = (int32_t)(b / g.ntail_x), i = (int32_t)(b % g.ntail_x);
      const int32_t x = x0 + 2 * i;
      const uint8_t* yr = frame + (int64_t)(2 * j) * g.pitch + x;
      const uint8_t* c = uvp + (int64_t)j * g.pitch + x;
      const BlockK k = block_consts(c[0], c[1]);
      count_px(lds, yr[0], k, lane4);
      count_px(lds, yr[1], k, lane4);
      count_px(lds, yr[g.pitch], k, lane4);
      count_px(lds, yr[g.pitch + 1], k, lane4);
    }
  }
  __syncthreads();

  // Sum the 64 lane columns of every (channel, sub-bin) row; rotate the
  // starting lane per thread so that concurrent rows hit different banks.
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(lds);
  if (tid < 3 * kSub) {
    uint32_t acc = 0;
    for (int l = 0; l < 64; ++l) acc += tab[tid * 64 + ((l + tid) & 63)];
    part[tid] = acc;
  }
  __syncthreads();
  if (tid < 48) {
    const int c = tid >> 4, k = tid & 15;
    uint32_t acc = 0;
    const int lo = (k == 0) ? 0 : k + kSubBias;
    const int hi = (k == 15) ? kSub - 1 : k + kSubBias;
    for (int sb = lo; sb <= hi; ++sb) acc += part[c * kSub + sb];
    if (acc) atomicAdd(&hist[m * 48 + tid], acc);
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// conversion

__device__ __forceinline__ uint32_t clamp_q14(int s) {
  return (uint32_t)min(max(s >> 14, 0), 255);
}

struct Rgb {
  uint32_t r, g, b;
};

// Per-block chroma terms of the Q14 sums (the +8192 rounding and -16 luma
// offset folded in) and the per-pixel completion.
struct BlockC {
  int r, g, b;
};
__device__ __forceinline__ BlockC chroma_terms(uint32_t u, uint32_t v) {
  const int uu = (int)u - 128, vv = (int)v - 128;
  BlockC c;
  c.r = cRV * vv + 8192 - 16 * cY;
  c.g = -cGU * uu - cGV * vv + 8192 - 16 * cY;
  c.b = cBU * uu + 8192 - 16 * cY;
  return c;
}
__device__ __forceinline__ Rgb to_rgb(uint32_t y, const BlockC& c) {
  const int ty = (int)y * cY;
  return Rgb{clamp_q14(ty + c.r), clamp_q14(ty + c.g), clamp_q14(ty + c.b)};
}

// 4x-scaled chroma terms for the vector path: t = 4 s keeps the channel in
// byte 2 once clamped to [0, 2^24), so no shift is needed before packing.
__device__ __forceinline__ BlockC chroma_terms4(uint32_t u, uint32_t v) {
  const BlockC c = chroma_terms(u, v);
  return BlockC{4 * c.r, 4 * c.g, 4 * c.b};
}
__device__ __forceinline__ int clamp_t(int t) { return min(max(t, 0), 0xFFFFFF); }
// Dword of the bytes 2 of four t values (b0 lowest).
__device__ __forceinline__ uint32_t pack4(int b0, int b1, int b2, int b3) {
  return __builtin_amdgcn_perm((uint32_t)b1, (uint32_t)b0, 0x0C0C0602u) |
         __builtin_amdgcn_perm((uint32_t)b3, (uint32_t)b2, 0x06020C0Cu);
}

struct ConvGeom {
  const uint8_t* frames;
  int64_t frame_bytes;
  int32_t width, height, pitch;
  int32_t nseg_x, ntail_x;
};

// RGB24 at full resolution.  Vector path: one thread converts 16 x 2 pixels
// (3 x 16 B loads, 6 x 16 B stores).  Grid: (segments + tail blocks) per frame x M.
template <bool kVec>
__global__ void __launch_bounds__(kThreads) k_nv12_rgb24(ConvGeom g, const int64_t* __restrict__ rows,
                                                         uint8_t* __restrict__ out, int64_t units_per_frame,
                                                         int32_t blocks_per_frame) {
  const int64_t m = blockIdx.x / blocks_per_frame;
  const int64_t unit = (int64_t)(blockIdx.x % blocks_per_frame) * kThreads + threadIdx.x;
  if (unit >= units_per_frame) return;
  const uint8_t* frame = g.frames + rows[m] * g.frame_bytes;
  const uint8_t* uvp = frame + (int64_t)g.pitch * g.height;
  uint8_t* of = out + m * (int64_t)g.width * g.height * 3;
  const int64_t nseg = kVec ? (int64_t)g.nseg_x * (g.height >> 1) : 0;
  if (kVec && unit < nseg) {
    const int32_t j = (int32_t)(unit / g.nseg_x), i = (int32_t)(unit % g.nseg_x);
    const uint8_t* yr = frame + (int64_t)(2 * j) * g.pitch + 16 * i;
    const uint4 a0 = *reinterpret_cast<const uint4*>(yr);
    const uint4 a1 = *reinterpret_cast<const uint4*>(yr + g.pitch);
    const uint4 a2 = *reinterpret_cast<const uint4*>(uvp + (int64_t)j * g.pitch + 16 * i);
    const uint32_t Y0[4] = {a0.x, a0.y, a0.z, a0.w};
    const uint32_t Y1[4] = {a1.x, a1.y, a1.z, a1.w};
    const uint32_t UV[4] = {a2.x, a2.y, a2.z, a2.w};
    // Channel values as byte 2 of t = clamp(4 s, 0, 2^24 - 1) (= clamp(s >> 14, 0, 255)),
    // in output byte order R0 G0 B0 R1 ..., then packed with byte permutes.
    int t0[48], t1[48];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const BlockC c = chroma_terms4(byte_of(UV[d], 2 * h), byte_of(UV[d], 2 * h + 1));
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int b = 3 * (4 * d + 2 * h + e);  // byte offset of the pixel in the 48-byte row
          const int ty0 = (int)byte_of(Y0[d], 2 * h + e) * (4 * cY);
          const int ty1 = (int)byte_of(Y1[d], 2 * h + e) * (4 * cY);
          t0[b] = clamp_t(ty0 + c.r);
          t0[b + 1] = clamp_t(ty0 + c.g);
          t0[b + 2] = clamp_t(ty0 + c.b);
          t1[b] = clamp_t(ty1 + c.r);
          t1[b + 1] = clamp_t(ty1 + c.g);
          t1[b + 2] = clamp_t(ty1 + c.b);
        }
      }
    }
    uint32_t o0[12], o1[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      o0[k] = pack4(t0[4 * k], t0[4 * k + 1], t0[4 * k + 2], t0[4 * k + 3]);
      o1[k] = pack4(t1[4 * k], t1[4 * k + 1], t1[4 * k + 2], t1[4 * k + 3]);
    }
    uint4* d0 = reinterpret_cast<uint4*>(of + ((int64_t)(2 * j) * g.width + 16 * i) * 3);
    uint4* d1 = reinterpret_cast<uint4*>(of + ((int64_t)(2 * j + 1) * g.width + 16 * i) * 3);
    d0[0] = make_uint4(o0[0], o0[1], o0[2], o0[3]);
    d0[1] = make_uint4(o0[4], o0[5], o0[6], o0[7]);
    d0[2] = make_uint4(o0[8], o0[9], o0[10], o0[11]);
    d1[0] = make_uint4(o1[0], o1[1], o1[2], o1[3]);
    d1[1] = make_uint4(o1[4], o1[5], o1[6], o1[7]);
    d1[2] = make_uint4(o1[8], o1[9], o1[10], o1[11]);
    return;
  }
  // one 2x2 block
  const int64_t b = unit - nseg;
  const int32_t j = (int32_t)(b / g.ntail_x), i = (int32_t)(b % g.ntail_x);
  const int32_t x = 16 * (kVec ? g.nseg_x : 0) + 2 * i;
  const uint8_t* yr = frame + (int64_t)(2 * j) * g.pitch + x;
  const uint8_t* c = uvp + (int64_t)j * g.pitch + x;
  const BlockC cc = chroma_terms(c[0], c[1]);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const Rgb p = to_rgb(yr[r * g.pitch + e], cc);
      uint8_t* o = of + ((int64_t)(2 * j + r) * g.width + x + e) * 3;
      o[0] = (uint8_t)p.r;
      o[1] = (uint8_t)p.g;
      o[2] = (uint8_t)p.b;
    }
  }
}

// Bilinear tap of the resize (half-pixel centres, 8-bit weights).
struct Tap {
  int32_t i0, i1, f;
};
__device__ __forceinline__ Tap resize_tap(int32_t x, int32_t n_in, int32_t n_out) {
  int64_t n = (int64_t)(2 * x + 1) * n_in - n_out;
  if (n < 0) n = 0;
  const int64_t d = 2 * (int64_t)n_out;
  Tap t;
  t.i0 = (int32_t)min<int64_t>(n / d, n_in - 1);
  t.f = (int32_t)((256 * (n % d) + n_out) / d);
  t.i1 = min(t.i0 + 1, n_in - 1);
  return t;
}

__device__ __forceinline__ Rgb rgb_at(const uint8_t* frame, const uint8_t* uvp, int32_t pitch, int32_t x, int32_t y) {
  const uint8_t* c = uvp + (int64_t)(y >> 1) * pitch + (x & ~1);
  return to_rgb(frame[(int64_t)y * pitch + x], chroma_terms(c[0], c[1]));
}

// Gather + convert + resize (RGB24) or luma + resize (GRAY8); one output
// pixel per thread.  Grid: ceil(out_w * out_h / 256) per frame x M.
template <bool kGray>
__global__ void __launch_bounds__(kThreads) k_nv12_resize(ConvGeom g, const int64_t* __restrict__ rows,
                                                          uint8_t* __restrict__ out, int32_t out_w, int32_t out_h,
                                                          int32_t blocks_per_frame) {
  const int64_t m = blockIdx.x / blocks_per_frame;
  const int64_t p = (int64_t)(blockIdx.x % blocks_per_frame) * kThreads + threadIdx.x;
  if (p >= (int64_t)out_w * out_h) return;
  const int32_t ox = (int32_t)(p % out_w), oy = (int32_t)(p / out_w);
  const uint8_t* frame = g.frames + rows[m] * g.frame_bytes;
  const uint8_t* uvp = frame + (int64_t)g.pitch * g.height;
  const Tap tx = resize_tap(ox, g.width, out_w);
  const Tap ty = resize_tap(oy, g.height, out_h);
  const int w00 = (256 - tx.f) * (256 - ty.f), w01 = tx.f * (256 - ty.f);
  const int w10 = (256 - tx.f) * ty.f, w11 = tx.f * ty.f;
  if (kGray) {
    const int v = w00 * frame[(int64_t)ty.i0 * g.pitch + tx.i0] + w01 * frame[(int64_t)ty.i0 * g.pitch + tx.i1] +
                  w10 * frame[(int64_t)ty.i1 * g.pitch + tx.i0] + w11 * frame[(int64_t)ty.i1 * g.pitch + tx.i1];
    out[m * (int64_t)out_w * out_h + p] = (uint8_t)((v + 32768) >> 16);
    return;
  }
  const Rgb a = rgb_at(frame, uvp, g.pitch, tx.i0, ty.i0);
  const Rgb b = rgb_at(frame, uvp, g.pitch, tx.i1, ty.i0);
  const Rgb c = rgb_at(frame, uvp, g.pitch, tx.i0, ty.i1);
  const Rgb d = rgb_at(frame, uvp, g.pitch, tx.i1, ty.i1);
  uint8_t* o = out + (m * (int64_t)out_w * out_h + p) * 3;
  o[0] = (uint8_t)((w00 * (int)a.r + w01 * (int)b.r + w10 * (int)c.r + w11 * (int)d.r + 32768) >> 16);
  o[1] = (uint8_t)((w00 * (int)a.g + w01 * (int)b.g + w10 * (int)c.g + w11 * (int)d.g + 32768) >> 16);
  o[2] = (uint8_t)((w00 * (int)a.b + w01 * (int)b.b + w10 * (int)c.b + w11 * (int)d.b + 32768) >> 16);
}

// GRAY8 at full resolution: copy the sampled rows' luma planes.
__global__ void __launch_bounds__(kThreads) k_luma_copy(ConvGeom g, const int64_t* __restrict__ rows,
                                                        uint8_t* __restrict__ out, int32_t blocks_per_frame) {
  const int64_t m = blockIdx.x / blocks_per_frame;
  const int64_t p = (int64_t)(blockIdx.x % blocks_per_frame) * kThreads + threadIdx.x;
  const int64_t npx = (int64_t)g.width * g.height;
  if (p >= npx) return;
  const int32_t x = (int32_t)(p % g.width), y = (int32_t)(p / g.width);
  out[m * npx + p] = g.frames[rows[m] * g.frame_bytes + (int64_t)y * g.pitch + x];
}

// Shot-boundary cue: the L1 distance of the [3][16] histograms of the two
// sampled rows of each S[0,1] pair (Sec. 5.2.3 finds shot boundaries from
// histogram differences), and the cut flag d > threshold.  One wave per
// pair: lane b < 48 takes bin b of both histograms and the 48 absolute
// differences are summed across the wave (an exact integer sum, below 2^32
// because the host bounds the frame area).
__global__ void __launch_bounds__(256) k_hist_diff(const uint32_t* __restrict__ hist,
                                                   const int32_t* __restrict__ slots, int64_t n_pairs,
                                                   uint32_t threshold, uint32_t* __restrict__ diff,
                                                   uint8_t* __restrict__ cut) {
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= n_pairs) return;
  const int64_t i = slots[2 * p], j = slots[2 * p + 1];
  uint32_t d = 0;
  if (lane < 48) {
    const uint32_t a = hist[i * 48 + lane], b = hist[j * 48 + lane];
    d = a > b ? a - b : b - a;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d += (uint32_t)__shfl_xor((int)d, o, 64);
  if (lane == 0) {
    diff[p] = d;
    if (cut) cut[p] = d > threshold ? 1 : 0;
  }
}

bool vec_ok(const scn_table& t) {
  return ((uintptr_t)t.frames % 16 == 0) && (t.pitch % 16 == 0) && (t.frame_bytes % 16 == 0) && t.width >= 16;
}

}  // namespace

scn_status launch_hist(const scn_table& t, const int64_t* rows_dev, int64_t m, uint32_t* hist, hipStream_t s) {
  const int64_t n = m * 48;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, hist, n);
  SCN_LAUNCHED("hist zero launch");
  FrameGeom g;
  g.frames = t.frames;
  g.frame_bytes = t.frame_bytes;
  g.width = t.width;
  g.height = t.height;
  g.pitch = t.pitch;
  const bool vec = vec_ok(t);
  g.nseg_x = vec ? t.width / 16 : 0;
  g.ntail_x = (t.width - 16 * g.nseg_x) / 2;
  // about 16 segments (512 pixels) per thread per workgroup (the per-workgroup
  // clearing and folding of the LDS counters is then a small share)
  const int64_t px = (int64_t)t.width * t.height;
  g.chunks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(4096, px / (kThreads * 512)));
  const int64_t grid = m * g.chunks;
  if (grid > 0x7FFFFFFF) { set_error("too many frames for one HIST launch"); return SCN_EUNSUPPORTED; }
  KernelTimer timer("hist16", s);
  if (vec)
    hipLaunchKernelGGL(k_hist16<true>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, hist);
  else
    hipLaunchKernelGGL(k_hist16<false>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, hist);
  SCN_LAUNCHED("hist launch");
  return SCN_OK;
}

scn_status launch_hist_diff(const uint32_t* hist, const int32_t* slots_dev, int64_t n_pairs, uint32_t threshold,
                            uint32_t* diff, uint8_t* cut, hipStream_t s) {
  const int64_t grid = (n_pairs + 3) / 4;
  if (grid > 0x7FFFFFFF) { set_error("too many pairs for one launch"); return SCN_EUNSUPPORTED; }
  KernelTimer timer("hist_diff", s);
  hipLaunchKernelGGL(k_hist_diff, dim3((unsigned)grid), dim3(256), 0, s, hist, slots_dev, n_pairs, threshold, diff,
                     cut);
  SCN_LAUNCHED("hist diff launch");
  return SCN_OK;
}

scn_status launch_convert(const scn_table& t, const int64_t* rows_dev, int64_t m, int32_t out_w, int32_t out_h,
                          int32_t fmt, uint8_t* out, hipStream_t s) {
  ConvGeom g;
  g.frames = t.frames;
  g.frame_bytes = t.frame_bytes;
  g.width = t.width;
  g.height = t.height;
  g.pitch = t.pitch;
  const bool same = (out_w == t.width && out_h == t.height);
  if (fmt == SCN_RGB24 && same) {
    const bool vec = vec_ok(t) && ((uintptr_t)out % 16 == 0) && (t.width % 16 == 0);
    g.nseg_x = vec ? t.width / 16 : 0;
    g.ntail_x = (t.width - 16 * g.nseg_x) / 2;
    const int64_t units = (int64_t)(g.nseg_x + g.ntail_x) * (t.height / 2);
    const int64_t bpf = (units + kThreads - 1) / kThreads;
    const int64_t grid = m * bpf;
    if (grid > 0x7FFFFFFF) { set_error("too many frames for one convert launch"); return SCN_EUNSUPPORTED; }
    KernelTimer timer("nv12_rgb24", s);
    if (vec)
      hipLaunchKernelGGL(k_nv12_rgb24<true>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, out, units,
                         (int32_t)bpf);
    else
      hipLaunchKernelGGL(k_nv12_rgb24<false>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, out, units,
                         (int32_t)bpf);
    SCN_LAUNCHED("convert launch");
    return SCN_OK;
  }
  g.nseg_x = 0;
  g.ntail_x = 0;
  if (fmt == SCN_GRAY8 && same) {
    const int64_t bpf = ((int64_t)t.width * t.height + kThreads - 1) / kThreads;
    const int64_t grid = m * bpf;
    if (grid > 0x7FFFFFFF) { set_error("too many frames for one convert launch"); return SCN_EUNSUPPORTED; }
    KernelTimer timer("luma_copy", s);
    hipLaunchKernelGGL(k_luma_copy, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, out, (int32_t)bpf);
    SCN_LAUNCHED("luma copy launch");
    return SCN_OK;
  }
  const int64_t bpf = ((int64_t)out_w * out_h + kThreads - 1) / kThreads;
  const int64_t grid = m * bpf;
  if (grid > 0x7FFFFFFF) { set_error("too many frames for one resize launch"); return SCN_EUNSUPPORTED; }
  KernelTimer timer("nv12_resize", s);
  if (fmt == SCN_GRAY8)
    hipLaunchKernelGGL(k_nv12_resize<true>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, out, out_w,
                       out_h, (int32_t)bpf);
  else
    hipLaunchKernelGGL(k_nv12_resize<false>, dim3((unsigned)grid), dim3(kThreads), 0, s, g, rows_dev, out, out_w,
                       out_h, (int32_t)bpf);
  SCN_LAUNCHED("resize launch");
  return SCN_OK;
}

}  // namespace scn
