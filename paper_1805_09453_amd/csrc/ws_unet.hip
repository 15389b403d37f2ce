// Learned warm start for the EMD iteration: a 4-level U-Net that predicts the
// dual potential phi0 from (rho0, rho1), with hand-written BF16 MFMA kernels
// for inference and training on gfx950.
//
// The network and its parameter blob are described in include/gprox.h (and the
// warm-start section of the design notes): 3x3 conv + ReLU pairs with widths
// 32/64/128/256, 2x2 average pooling, 2x2 stride-2 transposed convolutions,
// skip concatenation [upsampled, skip], 1x1 head.  It is not part of the paper:
// the iteration it seeds is Algorithm 2 with the updates of section 3.2, whose
// duality gap still decides convergence.
//
// Layout: activations are NHWC BF16 (channels innermost, 8-channel 16-byte
// vectors); the FP32 master parameters, their gradients and the Adam moments
// live in flat blobs; each step regenerates BF16 packed copies of the weights
// in the [n][k] forms the GEMM kernels read.
//
// Kernels:
//   k_conv   implicit GEMM on v_mfma_f32_16x16x32_bf16: M = pixels (128 per
//            block), N = output channels (32 or 64 per block), K = taps x
//            input channels (32 per step, double-buffered in LDS).  Modes:
//            3x3 convolution (forward, and backward-data with flipped packed
//            weights), transposed-conv forward (N = 4 x cout, pixel-shuffle
//            store) and backward-data (K gathers the 2x2 output block).
//   k_wgrad  weight gradients as D[m][k] = sum_p A[p][m] B[p][k] with the
//            pixel sum split over blocks (FP32 atomics into the blob);
//            pixel-major operand tiles loaded straight into LDS, MFMA
//            fragments read with transposing LDS reads.
//   elementwise: input packing, pooling, ReLU and skip backward, head, loss,
//            channel sums (bias gradients), Adam, weight packing, resampling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gprox.h"
#include "ws_unet.hpp"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 ld16(const bf16* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st16(bf16* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }
__device__ __forceinline__ float b2f(bf16 x) { return float(x); }
__device__ __forceinline__ bf16 f2b(float x) { return bf16(x); }

union V8 {
  uint4 u;
  bf16 h[8];
};

// Workgroups go to the 8 XCDs round-robin (block b runs on XCD b mod 8), each
// XCD with its own L2.  This renumbering gives every XCD a contiguous range of
// [0, nb), so blocks that read the same pixels run under one L2.
__device__ __forceinline__ int xcd_range(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------ implicit-GEMM convolution
enum { M_CONV3 = 0, M_TFWD = 1, M_TBWD = 2 };

struct ConvArgs {
  const bf16* x1;  // first source (NHWC), c1 channels at stride s1 per pixel
  const bf16* x2;  // second source (concatenated after x1), nullable
  const bf16* w;   // packed weights [npad][kpad]
  const float* bias;
  bf16* y;
  int c1, s1, c2, s2;
  int B, H, W;    // GEMM pixel space: output pixels (conv), input pixels (transposed modes)
  int kpad, n;    // padded K; valid output channels N
  int ys, bmod;   // output pixel stride; bias index = n % bmod
  int relu;
};

// 16 zero bytes in device memory: the source of the operand pieces that lie
// outside the image or the padded K range (loads go straight to LDS, where no
// value can be masked)
__device__ __align__(16) uint4 g_zero16 = {0u, 0u, 0u, 0u};

// Address of 8 consecutive K entries (from k0) of row p of the implicit A matrix,
// with the pixel given as (b, y, x) and k0 as (tap, ci), k0 = tap ct + ci (3x3: ct =
// c1 + c2, tap = 3 dy + dx; transposed backward: ct = c1, the 2x2 output block): the
// K loop keeps these without integer divisions.  pin: p lies in the pixel space.
// Entries outside the image or the padded K range read g_zero16.
template <int MODE>
__device__ __forceinline__ const bf16* conv_a_src(const ConvArgs& a, bool pin, size_t p, int b, int y, int x, int k0,
                                                  int tap, int ci) {
  const bf16* zero = reinterpret_cast<const bf16*>(&g_zero16);
  if (!pin) return zero;
  if (MODE == M_CONV3) {
    if (tap >= 9) return zero;
    const int dy = (tap >= 3) + (tap >= 6), dx = tap - 3 * dy;
    const int yy = y + dy - 1, xx = x + dx - 1;
    if (yy < 0 || yy >= a.H || xx < 0 || xx >= a.W) return zero;
    // the neighbour is pixel p + (dy - 1) W + (dx - 1) of the same image
    const long long q = (long long)p + (dy - 1) * a.W + (dx - 1);
    return ci < a.c1 ? a.x1 + q * a.s1 + ci : a.x2 + q * a.s2 + (ci - a.c1);
  } else if (MODE == M_TFWD) {
    if (k0 >= a.c1) return zero;
    return a.x1 + p * a.s1 + k0;
  } else {
    if (tap >= 4) return zero;
    const size_t q = (size_t(b) * 2 * a.H + 2 * y + (tap >> 1)) * size_t(2 * a.W) + 2 * x + (tap & 1);
    return a.x1 + q * a.s1 + ci;
  }
}

// 16 bytes per lane from global memory straight into LDS: lane i's bytes land at
// lds + 16 i (lds is the same for the whole wave)
__device__ __forceinline__ void ld16_lds(const bf16* src, bf16* lds) {
  __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (__attribute__((address_space(3))) void*)(lds), 16,
                                   0, 0);
}

template <int MODE, int NT>
__global__ __launch_bounds__(256, NT == 32 ? 7 : 5) void k_conv(ConvArgs a) {
  // LDS tiles [row][KS] without padding; the four 16-byte chunks of row r are
  // stored in the order chunk ^ ((r / 2) mod 4), so that the MFMA operand reads
  // (eight rows per eight lanes) are free of bank conflicts
  constexpr int MT = 128, KS = 32, LD = KS;
  // two buffers per operand, as separate objects: the compiler can then tell the
  // reads of one from the loads into the other and does not wait for those loads
  __shared__ __align__(16) bf16 As0[MT * LD], As1[MT * LD];
  __shared__ __align__(16) bf16 Bs0[NT * LD], Bs1[NT * LD];
  auto tl = [](int row, int chunk) { return row * LD + ((chunk ^ ((row >> 1) & 3)) << 3); };
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the channel tiles of one pixel tile are consecutive blocks of one XCD (they
  // gather the same activations)
  const int gy = gridDim.y, lb = xcd_range(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gy);
  const int p0 = (lb / gy) * MT, n0 = (lb - (lb / gy) * gy) * NT;
  const int M = a.B * a.H * a.W;
  const int nsteps = a.kpad / KS;
  // the operand pieces go from global memory straight into LDS, 16 bytes per lane
  // at the lane's slot of the tile: thread tid fills slot tid % 4 of A rows tid / 4
  // and 64 + tid / 4 (pixels p0 + row) and, below 4 NT threads, of B row tid / 4.
  // The slot holds logical K chunk lc of the step (the swizzle of the row), so the
  // thread loads K offset lc * 8 + s KS.
  const int lc = (tid & 3) ^ ((tid >> 3) & 3);
  int pb_[2], py_[2], px_[2];
  bool pin[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int p = p0 + ((tid + 256 * j) >> 2);
    const int hw = a.H * a.W;
    pin[j] = p < M;
    pb_[j] = p / hw;
    const int r = p - pb_[j] * hw;
    py_[j] = r / a.W;
    px_[j] = r - py_[j] * a.W;
  }
  const int ct = max(1, MODE == M_CONV3 ? a.c1 + a.c2 : a.c1);
  int ktap = (lc * 8) / ct, kci = lc * 8 - ktap * ct;
  // 3x3 layers whose source widths are multiples of KS (all but the input layer):
  // every K step is one tap of one source for the whole block, so the tap, its
  // pixel offset and the source are uniform; per thread only a precomputed
  // pixel offset per source and a mask of the taps that stay inside the image
  const bool uni = MODE == M_CONV3 && a.c1 % KS == 0 && a.c2 % KS == 0;
  int utap = 0, ucib = 0;
  long long o1[2] = {0, 0}, o2[2] = {0, 0};
  unsigned tmask[2] = {0u, 0u};
  if (uni) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long long p = p0 + ((tid + 256 * j) >> 2);
      o1[j] = p * a.s1;
      o2[j] = p * a.s2;
      for (int t = 0; t < 9; ++t) {
        const int yy = py_[j] + t / 3 - 1, xx = px_[j] + t % 3 - 1;
        if (pin[j] && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) tmask[j] |= 1u << t;
      }
    }
  }
  const bf16* zero = reinterpret_cast<const bf16*>(&g_zero16);
  // issues step s's loads into the LDS buffers Ab, Bb; called for s = 0, 1, 2, ... in turn
  auto gload = [&](int s, bf16* Ab, bf16* Bb) {
    if (uni) {
      const int dy = (utap >= 3) + (utap >= 6), dx = utap - 3 * dy;
      const bool first = ucib < a.c1;
      const bf16* base = first ? a.x1 : a.x2;
      const long long toff = (long long)((dy - 1) * a.W + (dx - 1)) * (first ? a.s1 : a.s2) +
                             (first ? ucib : ucib - a.c1) + lc * 8;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bool ok = (tmask[j] >> utap) & 1u;
        ld16_lds(ok ? base + (first ? o1[j] : o2[j]) + toff : zero, Ab + (j * 256 + w * 64) * 8);
      }
      ucib += KS;
      if (ucib >= ct) {
        ucib = 0;
        ++utap;
      }
    } else {
      const int k0 = s * KS + lc * 8;
#pragma unroll
      for (int j = 0; j < 2; ++j)
        ld16_lds(conv_a_src<MODE>(a, pin[j], size_t(p0 + ((tid + 256 * j) >> 2)), pb_[j], py_[j], px_[j], k0, ktap,
                                  kci),
                 Ab + (j * 256 + w * 64) * 8);
      kci += KS;
      while (kci >= ct) {
        kci -= ct;
        ++ktap;
      }
    }
    if (tid < NT * 4)  // whole waves
      ld16_lds(a.w + size_t(n0 + (tid >> 2)) * a.kpad + s * KS + lc * 8, Bb + w * 64 * 8);
  };
  f32x4 acc[2][NT / 16];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT / 16; ++ni) acc[mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};
  // step s multiplies the operands in (Ar, Br) while step s + 1's load into (Aw, Bw),
  // which were last read before the previous barrier
  auto step = [&](int s, const bf16* Ar, const bf16* Br, bf16* Aw, bf16* Bw) {
    if (s + 1 < nsteps) gload(s + 1, Aw, Bw);
    bf16x8 bv[NT / 16];
#pragma unroll
    for (int ni = 0; ni < NT / 16; ++ni)
      bv[ni] = *reinterpret_cast<const bf16x8*>(&Br[tl(ni * 16 + (lane & 15), lane >> 4)]);
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&Ar[tl(w * 32 + mi * 16 + (lane & 15), lane >> 4)]);
      // weights as the first operand: the accumulator of lane l holds output
      // channels 4 (l / 16) + i, i < 4, of pixel l mod 16 of the 16 x 16 tile
#pragma unroll
      for (int ni = 0; ni < NT / 16; ++ni)
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bv[ni], av, acc[mi][ni], 0, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next buffers' loads have landed
    __syncthreads();
  };
  gload(0, As0, Bs0);
  __builtin_amdgcn_s_waitcnt(0);  // the LDS-bound loads have landed
  __syncthreads();
  for (int s = 0; s < nsteps; s += 2) {
    step(s, As0, Bs0, As1, Bs1);
    if (s + 1 < nsteps) step(s + 1, As1, Bs1, As0, Bs0);
  }
  // epilogue: bias, ReLU, BF16; each lane stores its 4 consecutive channels of a
  // pixel as one 8-byte vector (channel counts are multiples of 8)
  float bias[NT / 16][4];
#pragma unroll
  for (int ni = 0; ni < NT / 16; ++ni) {
    const int n = n0 + ni * 16 + 4 * (lane >> 4);
    const int nb = a.bias && n < a.n ? n % a.bmod : -1;  // n and bmod are multiples of 4
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[ni][i] = nb >= 0 ? a.bias[nb + i] : 0.f;
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi) {
    const int p = p0 + w * 32 + mi * 16 + (lane & 15);
    if (p >= M) continue;
    // transposed forward: output pixel (2y + tap / 2, 2x + tap % 2) of the 2x2 block
    size_t qb = 0;
    if (MODE == M_TFWD) {
      const int hw = a.H * a.W, b = p / hw, r = p - b * hw, y = r / a.W, x = r - y * a.W;
      qb = (size_t(b) * 2 * a.H + 2 * y) * size_t(2 * a.W) + 2 * x;
    }
#pragma unroll
    for (int ni = 0; ni < NT / 16; ++ni) {
      const int n = n0 + ni * 16 + 4 * (lane >> 4);
      if (n >= a.n) continue;
      unsigned short h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = acc[mi][ni][i] + bias[ni][i];
        if (a.relu) v = fmaxf(v, 0.f);
        h[i] = __builtin_bit_cast(unsigned short, f2b(v));
      }
      const uint2 val = make_uint2(uint32_t(h[0]) | (uint32_t(h[1]) << 16), uint32_t(h[2]) | (uint32_t(h[3]) << 16));
      bf16* dst;
      if (MODE == M_TFWD) {
        const int cout = a.bmod, tap = n / cout, co = n - tap * cout;
        dst = a.y + (qb + size_t(tap >> 1) * size_t(2 * a.W) + (tap & 1)) * a.ys + co;
      } else {
        dst = a.y + size_t(p) * a.ys + n;
      }
      *reinterpret_cast<uint2*>(dst) = val;
    }
  }
}

// ------------------------------------------------------------ weight gradients
enum { W_CONV3 = 0, W_TCONV = 1 };

struct WgArgs {
  const bf16* t1;  // m-operand tensor (c1m channels at stride s1m)
  const bf16* x1;  // k-operand sources (as ConvArgs)
  const bf16* x2;
  float* dw;       // FP32 blob slice, dst = (m * taps + tap) * ckeep + c
  int c1m, s1m;
  int c1, s1, c2, s2;
  int B, H, W;     // pixel space of the m-operand
  int taps, ck, ckeep;
  int chunk;       // pixels per block (multiple of 64)
};

// Address of 8 consecutive k entries of the k operand at pixel (b, y, x), k = tap ck +
// c.  Entries outside the image or past the taps are zero: ok is false (and the
// address the first vector of x1); the caller then reads the zero vector instead.
template <int MODE>
__device__ __forceinline__ const bf16* wg_k_src(const WgArgs& a, int b, int y, int x, int tap, int c, bool& ok) {
  if (MODE == W_CONV3) {
    const int t = tap < a.taps ? tap : 0;
    const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
    ok = tap < a.taps && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
    const size_t q = ok ? (size_t(b) * a.H + yy) * a.W + xx : 0;
    const bf16* src = c < a.c1 ? a.x1 + q * a.s1 + c : a.x2 + q * a.s2 + (c - a.c1);
    return ok ? src : a.x1;
  } else {
    ok = tap < a.taps;
    const size_t q = (size_t(b) * 2 * a.H + 2 * y + (tap >> 1)) * size_t(2 * a.W) + 2 * x + (tap & 1);
    return ok ? a.x1 + q * a.s1 + c : a.x1;
  }
}

typedef short s16x4 __attribute__((ext_vector_type(4)));
// gfx950 transposing LDS read: in each group of 16 lanes whose addresses cover a
// 4 x 16 block of 16-bit values (lane j: row j / 4, columns 4 (j mod 4) .. + 3),
// lane i receives column i of the four rows
__device__ __forceinline__ s16x4 ld_tr16(const bf16* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)(p));
}

template <int MODE>
__global__ __launch_bounds__(256, 5) void k_wgrad(WgArgs a) {
  // Tiles of 64 pixels per step, pixel-major as in memory: At[p][m] (64 m
  // channels) and Bt[p][k] (64 k entries), 128-byte rows whose 16-byte chunks are
  // stored in the order chunk ^ 2 (p mod 4).  Both are loaded straight into LDS
  // (16 bytes per lane; pieces outside the image, the taps or the channels read a
  // zero vector), double-buffered as separate LDS objects with the loop unrolled by
  // two, so the loads of the next step overlap this step's MFMAs.  The MFMA
  // fragments (8 consecutive pixels of one channel per lane) are two transposing
  // reads of 4 x 16 blocks each; with the chunk order above these are free of bank
  // conflicts.  Wave w computes m rows 16 w .. + 16 of the 64 x 64 (m, k) tile.
  constexpr int PS = 64, TS = PS * 64;
  __shared__ __align__(16) bf16 At0[TS], At1[TS], Bt0[TS], Bt1[TS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the (m, k) tiles of one pixel chunk are consecutive blocks of one XCD (they
  // read the same pixels)
  const int gx = gridDim.x, gxy = gx * gridDim.y;
  const int lb = xcd_range(blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z), gxy * gridDim.z);
  const int bz = lb / gxy, by = (lb - bz * gxy) / gx, bx = lb - bz * gxy - by * gx;
  const int m0 = bx * 64, k0 = by * 64;
  const int P = a.B * a.H * a.W;
  const int pb = bz * a.chunk, pe = min(P, pb + a.chunk);
  f32x4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this thread's two pieces of a step: pixel rows pr[j] = 32 j + 8 w + lane / 8 of
  // the tile, physical chunk lane % 8, holding logical chunk lc (channels / k
  // entries 8 lc .. + 7); the LDS slot of piece j is 16 (256 j + tid) bytes
  const int lc = (lane & 7) ^ (2 * ((lane >> 3) & 3));
  const bool mok = m0 + 8 * lc < a.c1m;
  const int ktap = (k0 + 8 * lc) / a.ck, kc = (k0 + 8 * lc) - ktap * a.ck;
  const bool wact = m0 + w * 16 < a.c1m;
  const bf16* zero = reinterpret_cast<const bf16*>(&g_zero16);
  // (b, y, x) of each piece's pixel, moved on by whole steps without divisions
  int cb[2], cy[2], cx[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int p = pb + 32 * j + 8 * w + (lane >> 3), hw = a.H * a.W;
    cb[j] = p / hw;
    const int r = p - cb[j] * hw;
    cy[j] = r / a.W;
    cx[j] = r - cy[j] * a.W;
  }
  auto advance = [&]() {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cx[j] += PS;
      while (cx[j] >= a.W) {
        cx[j] -= a.W;
        if (++cy[j] == a.H) {
          cy[j] = 0;
          ++cb[j];
        }
      }
    }
  };
  // issues the loads of the step at pixel ps (the pixel state is at ps) into (Aw, Bw)
  auto gload = [&](int ps, bf16* Aw, bf16* Bw) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = ps + 32 * j + 8 * w + (lane >> 3);
      const bool in = p < pe;
      ld16_lds(in && mok ? a.t1 + size_t(p) * a.s1m + m0 + 8 * lc : zero, Aw + (256 * j + 64 * w) * 8);
      bool ok;
      const bf16* src = wg_k_src<MODE>(a, cb[j], cy[j], cx[j], ktap, kc, ok);
      ld16_lds(in && ok ? src : zero, Bw + (256 * j + 64 * w) * 8);
    }
  };
  // element offset of a transposing read's 8 bytes for lane i of its group: rows
  // rb + i / 4, logical columns cb0 + 4 (i mod 4) .. + 3
  auto tra = [](int rb, int cb0, int i) {
    const int row = rb + (i >> 2), col = cb0 + 4 * (i & 3);
    return row * 64 + ((((col >> 3) ^ (2 * (row & 3)))) << 3) + (col & 7);
  };
  auto step = [&](int ps, const bf16* Ar, const bf16* Br, bf16* Aw, bf16* Bw) {
    if (ps + PS < pe) {
      advance();
      gload(ps + PS, Aw, Bw);
    }
    if (wact) {
      const int g = lane >> 4, i = lane & 15;
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int rb = kk * 32 + 8 * g;
        const s16x4 a0 = ld_tr16(Ar + tra(rb, w * 16, i)), a1 = ld_tr16(Ar + tra(rb + 4, w * 16, i));
        const bf16x8 av = __builtin_bit_cast(bf16x8, __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          const s16x4 b0 = ld_tr16(Br + tra(rb, ni * 16, i)), b1 = ld_tr16(Br + tra(rb + 4, ni * 16, i));
          const bf16x8 bv = __builtin_bit_cast(bf16x8, __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
          acc[ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ni], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next buffers' loads have landed
    __syncthreads();
  };
  gload(pb, At0, Bt0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int ps = pb; ps < pe; ps += 2 * PS) {
    step(ps, At0, Bt0, At1, Bt1);
    if (ps + PS < pe) step(ps + PS, At1, Bt1, At0, Bt0);
  }
#pragma unroll
  for (int ni = 0; ni < 4; ++ni)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + w * 16 + (lane >> 4) * 4 + i, k = k0 + ni * 16 + (lane & 15);
      if (m >= a.c1m) continue;
      const int tap = k / a.ck, c = k - tap * a.ck;
      if (tap < a.taps && c < a.ckeep) atomicAdd(&a.dw[(size_t(m) * a.taps + tap) * a.ckeep + c], acc[ni][i]);
    }
}

// ------------------------------------------------------------ elementwise kernels
#define GRID_STRIDE(i, n) \
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < size_t(n); i += size_t(gridDim.x) * blockDim.x)

// x0[p] = (rho0 - 1, rho1 - 1, 0, ..., 0)  (8 channels)
__global__ void k_prep(const float* __restrict__ r0, const float* __restrict__ r1, size_t P, bf16* __restrict__ x0) {
  GRID_STRIDE(p, P) {
    V8 v;
    v.u = uint4{0u, 0u, 0u, 0u};
    v.h[0] = f2b(r0[p] - 1.f);
    v.h[1] = f2b(r1[p] - 1.f);
    st16(x0 + p * 8, v.u);
  }
}

// 2x2 average pooling, [B][H][W][C] -> [B][H/2][W/2][C]
__global__ void k_pool(const bf16* __restrict__ x, int B, int H, int W, int C, bf16* __restrict__ y) {
  const int Ho = H / 2, Wo = W / 2, cv = C / 8;
  const size_t n = size_t(B) * Ho * Wo * cv;
  GRID_STRIDE(i, n) {
    const int c8 = int(i % cv);
    const size_t po = i / cv;
    const int xo = int(po % Wo), yo = int((po / Wo) % Ho), b = int(po / (size_t(Wo) * Ho));
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        V8 v;
        v.u = ld16(x + ((size_t(b) * H + 2 * yo + dy) * W + 2 * xo + dx) * C + 8 * c8);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += b2f(v.h[j]);
      }
    V8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o.h[j] = f2b(0.25f * s[j]);
    st16(y + po * C + 8 * c8, o.u);
  }
}

// out[p][c] = dy[p * sdy + c] * (y[p * C + c] > 0)   (in place allowed when out == dy, sdy == C)
// (the network's channel counts are powers of two: the vector index splits by shifts)
__global__ void k_relu_bwd(const bf16* dy, int sdy, const bf16* __restrict__ y, size_t P, int C, bf16* out) {
  const int cv = C / 8, lcv = __builtin_ctz(unsigned(cv));
  GRID_STRIDE(i, P * cv) {
    const size_t p = i >> lcv;
    const int c = int(i & size_t(cv - 1)) * 8;
    V8 g, a, o;
    g.u = ld16(dy + p * sdy + c);
    a.u = ld16(y + p * C + c);
#pragma unroll
    for (int j = 0; j < 8; ++j) o.h[j] = b2f(a.h[j]) > 0.f ? g.h[j] : f2b(0.f);
    st16(out + p * C + c, o.u);
  }
}

// encoder skip tensor S ([B][H][W][C]) feeds the pooling and the decoder concat:
// out = (pool^T dpool + dcat[:, off:off+C]) * (S > 0)
__global__ void k_skip_bwd(const bf16* __restrict__ dpool, const bf16* __restrict__ dcat, int scat,
                           const bf16* __restrict__ S, int B, int H, int W, int C, bf16* __restrict__ out) {
  const int cv = C / 8, lcv = __builtin_ctz(unsigned(cv));  // C a power of two
  const size_t n = size_t(B) * H * W * cv;
  GRID_STRIDE(i, n) {
    const int c = int(i & size_t(cv - 1)) * 8;
    const size_t p = i >> lcv;
    // pixel coordinates in 32-bit arithmetic (B H W < 2^32 for any network size)
    const unsigned pu = unsigned(p), q = pu / unsigned(W);
    const int x = int(pu - q * unsigned(W)), y = int(q % unsigned(H)), b = int(q / unsigned(H));
    V8 gp, gc, s, o;
    gp.u = ld16(dpool + ((size_t(b) * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
    gc.u = ld16(dcat + p * scat + c);
    s.u = ld16(S + p * C + c);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      o.h[j] = b2f(s.h[j]) > 0.f ? f2b(0.25f * b2f(gp.h[j]) + b2f(gc.h[j])) : f2b(0.f);
    st16(out + p * C + c, o.u);
  }
}

// head: phi[p] = b + sum_c w[c] x[p][c]   (C = 32)
__global__ void k_head_fwd(const bf16* __restrict__ x, const float* __restrict__ w, const float* __restrict__ b,
                           size_t P, float* __restrict__ phi) {
  GRID_STRIDE(p, P) {
    float s = b[0];
#pragma unroll
    for (int c8 = 0; c8 < 4; ++c8) {
      V8 v;
      v.u = ld16(x + p * 32 + 8 * c8);
#pragma unroll
      for (int j = 0; j < 8; ++j) s += w[8 * c8 + j] * b2f(v.h[j]);
    }
    phi[p] = s;
  }
}

// head backward fused with the ReLU of its input: g[p][c] = dphi[p] w[c] (x > 0);
// dw[c] += sum_p dphi x[p][c], db += sum dphi
__global__ __launch_bounds__(256) void k_head_bwd(const bf16* __restrict__ x, const float* __restrict__ w,
                                                  const float* __restrict__ dphi, size_t P, bf16* __restrict__ g,
                                                  float* __restrict__ dw, float* __restrict__ db) {
  float aw[32], ab = 0.f;
#pragma unroll
  for (int c = 0; c < 32; ++c) aw[c] = 0.f;
  GRID_STRIDE(p, P) {
    const float d = dphi[p];
    ab += d;
#pragma unroll
    for (int c8 = 0; c8 < 4; ++c8) {
      V8 v, o;
      v.u = ld16(x + p * 32 + 8 * c8);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float xv = b2f(v.h[j]);
        aw[8 * c8 + j] += d * xv;
        o.h[j] = f2b(xv > 0.f ? d * w[8 * c8 + j] : 0.f);
      }
      st16(g + p * 32 + 8 * c8, o.u);
    }
  }
  __shared__ float red[33][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 33; ++c) {
    float v = c < 32 ? aw[c] : ab;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 33) {
    float v = 0.f;
    for (int q = 0; q < int(blockDim.x >> 6); ++q) v += red[threadIdx.x][q];
    atomicAdd(threadIdx.x < 32 ? &dw[threadIdx.x] : db, v);
  }
}

// bias gradient: out[c] += sum_p g[p * S + c]  (C = 32, 64, 128 or 256; S a multiple
// of 8): each thread sums one 16-byte vector of 8 channels over a strided set of
// pixels, then the block adds its partial sums per channel
__global__ __launch_bounds__(256) void k_chsum(const bf16* __restrict__ g, int C, int S, size_t P,
                                               float* __restrict__ out) {
  const int G = C / 8, per = 256 / G;  // vectors per pixel; pixels side by side
  const int q = threadIdx.x % G, r = threadIdx.x / G;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // four independent 16-byte loads in flight per thread and trip
  const size_t stride = size_t(gridDim.x) * per;
  size_t p = size_t(blockIdx.x) * per + r;
  for (; p + 3 * stride < P; p += 4 * stride) {
    V8 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u].u = ld16(g + (p + u * stride) * S + 8 * q);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += b2f(v[u].h[j]);
  }
  for (; p < P; p += stride) {
    V8 v;
    v.u = ld16(g + p * S + 8 * q);
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += b2f(v.h[j]);
  }
  __shared__ float red[256 * 8];
#pragma unroll
  for (int j = 0; j < 8; ++j) red[threadIdx.x * 8 + j] = s[j];
  __syncthreads();
  if (int(threadIdx.x) < C) {
    const int c = threadIdx.x, cq = c / 8, cj = c % 8;
    float v = 0.f;
    for (int rr = 0; rr < per; ++rr) v += red[(rr * G + cq) * 8 + cj];
    atomicAdd(&out[c], v);
  }
}

// loss = sum |grad_h phi - grad_h phi*|^2 (added to *loss) and dphi = (2/N) grad_h^T e
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ phi, const float* __restrict__ st, int B,
                                              int ny, int nx, double inv_h, double inv_N, float* __restrict__ dphi,
                                              double* __restrict__ loss) {
  const size_t n = size_t(ny) * nx, P = n * B;
  double acc = 0.0;
  auto ex = [&](size_t base, int i, int j) -> double {  // x-component of e at (i, j)
    if (j < 0 || j >= nx - 1) return 0.0;
    const size_t o = base + size_t(i) * nx + j;
    return inv_h * ((double(phi[o + 1]) - phi[o]) - (double(st[o + 1]) - st[o]));
  };
  auto ey = [&](size_t base, int i, int j) -> double {
    if (i < 0 || i >= ny - 1) return 0.0;
    const size_t o = base + size_t(i) * nx + j;
    return inv_h * ((double(phi[o + nx]) - phi[o]) - (double(st[o + nx]) - st[o]));
  };
  GRID_STRIDE(o, P) {
    const size_t base = (o / n) * n, r = o - base;
    const int i = int(r / nx), j = int(r - size_t(i) * nx);
    const double a = ex(base, i, j), c = ey(base, i, j);
    acc += a * a + c * c;
    dphi[o] = float(2.0 * inv_N * inv_h * ((ex(base, i, j - 1) - a) + (ey(base, i - 1, j) - c)));
  }
  __shared__ double red[4];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int q = 0; q < int(blockDim.x >> 6); ++q) v += red[q];
    atomicAdd(loss, v);
  }
}

// a1 = 1 - b1 and a2 = 1 - b2 come from the host in FP64 (1.f - 0.999f is 1.3e-5 off)
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float a1, float a2, float eps,
                       float c1, float c2) {
  GRID_STRIDE(i, n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + a1 * gi;
    const float vi = b2 * v[i] + a2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_pack(const float* __restrict__ blob, const int* __restrict__ idx, size_t n, bf16* __restrict__ out) {
  GRID_STRIDE(i, n) {
    const int j = idx[i];
    out[i] = f2b(j >= 0 ? blob[j] : 0.f);
  }
}

__global__ void k_fill(float* __restrict__ p, size_t n) {
  GRID_STRIDE(i, n) p[i] = 0.f;
}
__global__ void k_fill64(double* p) { *p = 0.0; }

__global__ void k_down(const float* __restrict__ in, int ny, int nx, int f, float* __restrict__ out) {
  const int my = ny / f, mx = nx / f;
  GRID_STRIDE(o, size_t(my) * mx) {
    const int I = int(o / mx), J = int(o - size_t(I) * mx);
    float s = 0.f;
    for (int a = 0; a < f; ++a)
      for (int b = 0; b < f; ++b) s += in[size_t(I * f + a) * nx + J * f + b];
    out[o] = s / float(f * f);
  }
}

__global__ void k_up(const float* __restrict__ in, int ny, int nx, int f, float* __restrict__ out) {
  const int my = ny * f, mx = nx * f;
  GRID_STRIDE(o, size_t(my) * mx) {
    const int I = int(o / mx), J = int(o - size_t(I) * mx);
    const float yc = (I + 0.5f) / f - 0.5f, xc = (J + 0.5f) / f - 0.5f;
    const int y0 = int(floorf(yc)), x0 = int(floorf(xc));
    const float wy = yc - y0, wx = xc - x0;
    const int ya = min(max(y0, 0), ny - 1), yb = min(max(y0 + 1, 0), ny - 1);
    const int xa = min(max(x0, 0), nx - 1), xb = min(max(x0 + 1, 0), nx - 1);
    out[o] = (1.f - wy) * ((1.f - wx) * in[size_t(ya) * nx + xa] + wx * in[size_t(ya) * nx + xb]) +
             wy * ((1.f - wx) * in[size_t(yb) * nx + xa] + wx * in[size_t(yb) * nx + xb]);
  }
}

int gs(size_t n) {
  const size_t b = (n + 255) / 256;
  return int(b < 4096 ? (b ? b : 1) : 4096);
}

// ------------------------------------------------------------ network description
enum Kind { CONV3 = 0, TCONV2 = 1, HEAD = 2 };
struct Spec {
  int kind, cin, cout;
};
enum {
  L_E0A, L_E0B, L_E1A, L_E1B, L_E2A, L_E2B, L_MA, L_MB, L_U2, L_D2A, L_D2B, L_U1, L_D1A, L_D1B, L_U0, L_D0A, L_D0B,
  L_HEAD, L_COUNT
};
const Spec kSpecs[L_COUNT] = {{CONV3, 2, 32},    {CONV3, 32, 32},   {CONV3, 32, 64},    {CONV3, 64, 64},
                              {CONV3, 64, 128},  {CONV3, 128, 128}, {CONV3, 128, 256},  {CONV3, 256, 256},
                              {TCONV2, 256, 128}, {CONV3, 256, 128}, {CONV3, 128, 128}, {TCONV2, 128, 64},
                              {CONV3, 128, 64},  {CONV3, 64, 64},   {TCONV2, 64, 32},   {CONV3, 64, 32},
                              {CONV3, 32, 32},   {HEAD, 32, 1}};

int nt_for(int n) { return n % 64 == 0 ? 64 : 32; }
int rup(int x, int m) { return (x + m - 1) / m * m; }

struct Packed {  // one packed BF16 weight form: [npad][kpad]
  size_t off = 0;
  int n = 0, npad = 0, k = 0, kpad = 0;
};

struct Layer {
  Spec s;
  size_t woff = 0, boff = 0;  // offsets in the FP32 blob
  Packed fwd, bwd;
};

}  // namespace

struct ws_net {
  int B = 0, H = 0, W = 0;
  Layer L[L_COUNT];
  size_t nparam = 0, npacked = 0;
  float *par = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  bf16* packed = nullptr;
  int* pidx = nullptr;
  long long t = 0;
  double* loss_dev = nullptr;
  double* loss_host = nullptr;
  // activations (BF16 NHWC) and gradients
  bf16 *x0 = nullptr, *e0a, *s0, *p0, *e1a, *s1, *p1, *e2a, *s2, *p2, *ma, *mb, *u2, *d2a, *d2b, *u1, *d1a, *d1b,
       *u0, *d0a, *d0b;
  bf16 *g0a, *g0b, *dcat0, *dd1b, *g1a, *g1b, *dcat1, *dp0, *dd2b, *g2a, *g2b, *dcat2, *dp1, *dmb, *g3a, *g3b, *dp2;
  float *phi = nullptr, *dphi = nullptr;
  void* arena = nullptr;
  char err[256] = {0};
};

namespace {

void werr(ws_net* n, const char* msg, hipError_t e) {
  std::snprintf(n->err, sizeof(n->err), "%s: %s", msg, hipGetErrorString(e));
}

#define WCHK(net, call)                          \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) {                      \
      werr(net, #call, e_);                      \
      return GP_EHIP;                            \
    }                                            \
  } while (0)
#define WLAUNCH(net)                             \
  do {                                           \
    hipError_t e_ = hipGetLastError();           \
    if (e_ != hipSuccess) {                      \
      werr(net, "kernel launch", e_);            \
      return GP_EHIP;                            \
    }                                            \
  } while (0)

#define RCHK_(expr) \
  do {              \
    rc = (expr);    \
    if (rc) return rc; \
  } while (0)

// ---- GEMM launches
template <int MODE>
int launch_conv(ws_net* net, hipStream_t s, ConvArgs a, int npad) {
  const int M = a.B * a.H * a.W;
  const int nt = nt_for(npad);
  dim3 grid((M + 127) / 128, npad / nt);
  if (nt == 64)
    hipLaunchKernelGGL((k_conv<MODE, 64>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_conv<MODE, 32>), grid, dim3(256), 0, s, a);
  WLAUNCH(net);
  return GP_OK;
}

// y = act(conv3(x1 ++ x2)) over a B x H x W pixel space
int conv3_fwd(ws_net* net, hipStream_t s, int li, const bf16* x1, int c1, const bf16* x2, int c2, int B, int H,
              int W, bf16* y) {
  const Layer& l = net->L[li];
  ConvArgs a{};
  a.x1 = x1;
  a.c1 = c1;
  a.s1 = c1;
  a.x2 = x2;
  a.c2 = c2;
  a.s2 = c2;
  a.B = B;
  a.H = H;
  a.W = W;
  a.w = net->packed + l.fwd.off;
  a.kpad = l.fwd.kpad;
  a.n = l.s.cout;
  a.bias = net->par + l.boff;
  a.bmod = l.s.cout;
  a.relu = 1;
  a.y = y;
  a.ys = l.s.cout;
  return launch_conv<M_CONV3>(net, s, a, l.fwd.npad);
}

// dx = conv3^T(g): a conv of g with the flipped, transposed weights
int conv3_bwd_data(ws_net* net, hipStream_t s, int li, const bf16* g, int B, int H, int W, bf16* dx) {
  const Layer& l = net->L[li];
  ConvArgs a{};
  a.x1 = g;
  a.c1 = l.s.cout;
  a.s1 = l.s.cout;
  a.B = B;
  a.H = H;
  a.W = W;
  a.w = net->packed + l.bwd.off;
  a.kpad = l.bwd.kpad;
  a.n = l.bwd.n;
  a.bmod = 1;
  a.y = dx;
  a.ys = l.bwd.n;
  return launch_conv<M_CONV3>(net, s, a, l.bwd.npad);
}

int tconv_fwd(ws_net* net, hipStream_t s, int li, const bf16* x, int B, int H, int W, bf16* y) {
  const Layer& l = net->L[li];
  ConvArgs a{};
  a.x1 = x;
  a.c1 = l.s.cin;
  a.s1 = l.s.cin;
  a.B = B;
  a.H = H;
  a.W = W;
  a.w = net->packed + l.fwd.off;
  a.kpad = l.fwd.kpad;
  a.n = 4 * l.s.cout;
  a.bias = net->par + l.boff;
  a.bmod = l.s.cout;
  a.y = y;
  a.ys = l.s.cout;
  return launch_conv<M_TFWD>(net, s, a, l.fwd.npad);
}

// dx over the transposed conv's input pixels from dy (2H x 2W, cout channels at stride sdy)
int tconv_bwd_data(ws_net* net, hipStream_t s, int li, const bf16* dy, int sdy, int B, int H, int W, bf16* dx) {
  const Layer& l = net->L[li];
  ConvArgs a{};
  a.x1 = dy;
  a.c1 = l.s.cout;
  a.s1 = sdy;
  a.B = B;
  a.H = H;
  a.W = W;
  a.w = net->packed + l.bwd.off;
  a.kpad = l.bwd.kpad;
  a.n = l.s.cin;
  a.bmod = 1;
  a.y = dx;
  a.ys = l.s.cin;
  return launch_conv<M_TBWD>(net, s, a, l.bwd.npad);
}

template <int MODE>
int launch_wgrad(ws_net* net, hipStream_t s, WgArgs a) {
  const int P = a.B * a.H * a.W;
  const int mt = (a.c1m + 63) / 64, kt = (a.taps * a.ck + 63) / 64;
  int chunks = 2048 / (mt * kt);
  chunks = chunks < 1 ? 1 : chunks;
  const int maxc = (P + 255) / 256;
  chunks = chunks > maxc ? maxc : chunks;
  a.chunk = rup((P + chunks - 1) / chunks, 64);
  chunks = (P + a.chunk - 1) / a.chunk;
  hipLaunchKernelGGL((k_wgrad<MODE>), dim3(mt, kt, chunks), dim3(256), 0, s, a);
  WLAUNCH(net);
  return GP_OK;
}

int chsum(ws_net* net, hipStream_t s, const bf16* g, int C, int S, size_t P, float* out) {
  if (C < 8 || C > 256 || (C & (C - 1)) || S % 8) return GP_EINVAL;  // the network's widths are 32 ... 256
  const int per = 256 / (C / 8);  // pixels per block and step; about 16 steps per thread
  size_t blocks = (P + per * 16 - 1) / (per * 16);
  if (blocks > 512) blocks = 512;  // every block adds C atomics to the same C floats
  hipLaunchKernelGGL(k_chsum, dim3(blocks ? blocks : 1), dim3(256), 0, s, g, C, S, P, out);
  WLAUNCH(net);
  return GP_OK;
}

// gradients of a 3x3 conv layer from g = dL/d(pre-activation); dx (nullable) receives dL/dx
int conv3_bwd(ws_net* net, hipStream_t s, int li, const bf16* x1, int c1, const bf16* x2, int c2, const bf16* g,
              int B, int H, int W, bf16* dx) {
  const Layer& l = net->L[li];
  WgArgs a{};
  a.t1 = g;
  a.c1m = l.s.cout;
  a.s1m = l.s.cout;
  a.x1 = x1;
  a.c1 = c1;
  a.s1 = c1;
  a.x2 = x2;
  a.c2 = c2;
  a.s2 = c2;
  a.B = B;
  a.H = H;
  a.W = W;
  a.taps = 9;
  a.ck = c1 + c2;
  a.ckeep = l.s.cin;
  a.dw = net->grad + l.woff;
  int rc = launch_wgrad<W_CONV3>(net, s, a);
  if (!rc) rc = chsum(net, s, g, l.s.cout, l.s.cout, size_t(B) * H * W, net->grad + l.boff);
  if (!rc && dx) rc = conv3_bwd_data(net, s, li, g, B, H, W, dx);
  return rc;
}

// gradients of a transposed conv from dy (2H x 2W, stride sdy); dx receives dL/dx (H x W)
int tconv_bwd(ws_net* net, hipStream_t s, int li, const bf16* x, const bf16* dy, int sdy, int B, int H, int W,
              bf16* dx) {
  const Layer& l = net->L[li];
  WgArgs a{};
  a.t1 = x;
  a.c1m = l.s.cin;
  a.s1m = l.s.cin;
  a.x1 = dy;
  a.c1 = l.s.cout;
  a.s1 = sdy;
  a.B = B;
  a.H = H;
  a.W = W;
  a.taps = 4;
  a.ck = l.s.cout;
  a.ckeep = l.s.cout;
  a.dw = net->grad + l.woff;
  int rc = launch_wgrad<W_TCONV>(net, s, a);
  if (!rc) rc = chsum(net, s, dy, l.s.cout, sdy, size_t(B) * 4 * H * W, net->grad + l.boff);
  if (!rc) rc = tconv_bwd_data(net, s, li, dy, sdy, B, H, W, dx);
  return rc;
}

int relu_bwd(ws_net* net, hipStream_t s, const bf16* dy, int sdy, const bf16* y, size_t P, int C, bf16* out) {
  hipLaunchKernelGGL(k_relu_bwd, dim3(gs(P * C / 8)), dim3(256), 0, s, dy, sdy, y, P, C, out);
  WLAUNCH(net);
  return GP_OK;
}

int pool(ws_net* net, hipStream_t s, const bf16* x, int B, int H, int W, int C, bf16* y) {
  hipLaunchKernelGGL(k_pool, dim3(gs(size_t(B) * H * W * C / 32)), dim3(256), 0, s, x, B, H, W, C, y);
  WLAUNCH(net);
  return GP_OK;
}

int pack(ws_net* net, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(gs(net->npacked)), dim3(256), 0, s, net->par, net->pidx, net->npacked,
                     net->packed);
  WLAUNCH(net);
  return GP_OK;
}

int forward(ws_net* net, hipStream_t s, const float* r0, const float* r1, int B) {
  const int H = net->H, W = net->W;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  const size_t P0 = size_t(B) * H * W;
  hipLaunchKernelGGL(k_prep, dim3(gs(P0)), dim3(256), 0, s, r0, r1, P0, net->x0);
  WLAUNCH(net);
  int rc = conv3_fwd(net, s, L_E0A, net->x0, 8, nullptr, 0, B, H, W, net->e0a);
  if (!rc) rc = conv3_fwd(net, s, L_E0B, net->e0a, 32, nullptr, 0, B, H, W, net->s0);
  if (!rc) rc = pool(net, s, net->s0, B, H, W, 32, net->p0);
  if (!rc) rc = conv3_fwd(net, s, L_E1A, net->p0, 32, nullptr, 0, B, H1, W1, net->e1a);
  if (!rc) rc = conv3_fwd(net, s, L_E1B, net->e1a, 64, nullptr, 0, B, H1, W1, net->s1);
  if (!rc) rc = pool(net, s, net->s1, B, H1, W1, 64, net->p1);
  if (!rc) rc = conv3_fwd(net, s, L_E2A, net->p1, 64, nullptr, 0, B, H2, W2, net->e2a);
  if (!rc) rc = conv3_fwd(net, s, L_E2B, net->e2a, 128, nullptr, 0, B, H2, W2, net->s2);
  if (!rc) rc = pool(net, s, net->s2, B, H2, W2, 128, net->p2);
  if (!rc) rc = conv3_fwd(net, s, L_MA, net->p2, 128, nullptr, 0, B, H3, W3, net->ma);
  if (!rc) rc = conv3_fwd(net, s, L_MB, net->ma, 256, nullptr, 0, B, H3, W3, net->mb);
  if (!rc) rc = tconv_fwd(net, s, L_U2, net->mb, B, H3, W3, net->u2);
  if (!rc) rc = conv3_fwd(net, s, L_D2A, net->u2, 128, net->s2, 128, B, H2, W2, net->d2a);
  if (!rc) rc = conv3_fwd(net, s, L_D2B, net->d2a, 128, nullptr, 0, B, H2, W2, net->d2b);
  if (!rc) rc = tconv_fwd(net, s, L_U1, net->d2b, B, H2, W2, net->u1);
  if (!rc) rc = conv3_fwd(net, s, L_D1A, net->u1, 64, net->s1, 64, B, H1, W1, net->d1a);
  if (!rc) rc = conv3_fwd(net, s, L_D1B, net->d1a, 64, nullptr, 0, B, H1, W1, net->d1b);
  if (!rc) rc = tconv_fwd(net, s, L_U0, net->d1b, B, H1, W1, net->u0);
  if (!rc) rc = conv3_fwd(net, s, L_D0A, net->u0, 32, net->s0, 32, B, H, W, net->d0a);
  if (!rc) rc = conv3_fwd(net, s, L_D0B, net->d0a, 32, nullptr, 0, B, H, W, net->d0b);
  if (rc) return rc;
  const Layer& h = net->L[L_HEAD];
  hipLaunchKernelGGL(k_head_fwd, dim3(gs(P0)), dim3(256), 0, s, net->d0b, net->par + h.woff, net->par + h.boff, P0,
                     net->phi);
  WLAUNCH(net);
  return GP_OK;
}

int backward(ws_net* net, hipStream_t s, int B) {
  const int H = net->H, W = net->W;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  const size_t P0 = size_t(B) * H * W, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
  const Layer& h = net->L[L_HEAD];
  hipLaunchKernelGGL(k_head_bwd, dim3(gs(P0) < 1024 ? gs(P0) : 1024), dim3(256), 0, s, net->d0b, net->par + h.woff,
                     net->dphi, P0, net->g0b, net->grad + h.woff, net->grad + h.boff);
  WLAUNCH(net);
  int rc = GP_OK;
  // decoder level 0
  RCHK_(conv3_bwd(net, s, L_D0B, net->d0a, 32, nullptr, 0, net->g0b, B, H, W, net->g0a));
  RCHK_(relu_bwd(net, s, net->g0a, 32, net->d0a, P0, 32, net->g0a));
  RCHK_(conv3_bwd(net, s, L_D0A, net->u0, 32, net->s0, 32, net->g0a, B, H, W, net->dcat0));
  RCHK_(tconv_bwd(net, s, L_U0, net->d1b, net->dcat0, 64, B, H1, W1, net->dd1b));
  // decoder level 1
  RCHK_(relu_bwd(net, s, net->dd1b, 64, net->d1b, P1, 64, net->g1b));
  RCHK_(conv3_bwd(net, s, L_D1B, net->d1a, 64, nullptr, 0, net->g1b, B, H1, W1, net->g1a));
  RCHK_(relu_bwd(net, s, net->g1a, 64, net->d1a, P1, 64, net->g1a));
  RCHK_(conv3_bwd(net, s, L_D1A, net->u1, 64, net->s1, 64, net->g1a, B, H1, W1, net->dcat1));
  RCHK_(tconv_bwd(net, s, L_U1, net->d2b, net->dcat1, 128, B, H2, W2, net->dd2b));
  // decoder level 2
  RCHK_(relu_bwd(net, s, net->dd2b, 128, net->d2b, P2, 128, net->g2b));
  RCHK_(conv3_bwd(net, s, L_D2B, net->d2a, 128, nullptr, 0, net->g2b, B, H2, W2, net->g2a));
  RCHK_(relu_bwd(net, s, net->g2a, 128, net->d2a, P2, 128, net->g2a));
  RCHK_(conv3_bwd(net, s, L_D2A, net->u2, 128, net->s2, 128, net->g2a, B, H2, W2, net->dcat2));
  RCHK_(tconv_bwd(net, s, L_U2, net->mb, net->dcat2, 256, B, H3, W3, net->dmb));
  // bottleneck
  RCHK_(relu_bwd(net, s, net->dmb, 256, net->mb, P3, 256, net->g3b));
  RCHK_(conv3_bwd(net, s, L_MB, net->ma, 256, nullptr, 0, net->g3b, B, H3, W3, net->g3a));
  RCHK_(relu_bwd(net, s, net->g3a, 256, net->ma, P3, 256, net->g3a));
  RCHK_(conv3_bwd(net, s, L_MA, net->p2, 128, nullptr, 0, net->g3a, B, H3, W3, net->dp2));
  // encoder level 2
  hipLaunchKernelGGL(k_skip_bwd, dim3(gs(P2 * 128 / 8)), dim3(256), 0, s, net->dp2, net->dcat2 + 128, 256, net->s2,
                     B, H2, W2, 128, net->g2b);
  WLAUNCH(net);
  RCHK_(conv3_bwd(net, s, L_E2B, net->e2a, 128, nullptr, 0, net->g2b, B, H2, W2, net->g2a));
  RCHK_(relu_bwd(net, s, net->g2a, 128, net->e2a, P2, 128, net->g2a));
  RCHK_(conv3_bwd(net, s, L_E2A, net->p1, 64, nullptr, 0, net->g2a, B, H2, W2, net->dp1));
  // encoder level 1
  hipLaunchKernelGGL(k_skip_bwd, dim3(gs(P1 * 64 / 8)), dim3(256), 0, s, net->dp1, net->dcat1 + 64, 128, net->s1, B,
                     H1, W1, 64, net->g1b);
  WLAUNCH(net);
  RCHK_(conv3_bwd(net, s, L_E1B, net->e1a, 64, nullptr, 0, net->g1b, B, H1, W1, net->g1a));
  RCHK_(relu_bwd(net, s, net->g1a, 64, net->e1a, P1, 64, net->g1a));
  RCHK_(conv3_bwd(net, s, L_E1A, net->p0, 32, nullptr, 0, net->g1a, B, H1, W1, net->dp0));
  // encoder level 0
  hipLaunchKernelGGL(k_skip_bwd, dim3(gs(P0 * 32 / 8)), dim3(256), 0, s, net->dp0, net->dcat0 + 32, 64, net->s0, B,
                     H, W, 32, net->g0b);
  WLAUNCH(net);
  RCHK_(conv3_bwd(net, s, L_E0B, net->e0a, 32, nullptr, 0, net->g0b, B, H, W, net->g0a));
  RCHK_(relu_bwd(net, s, net->g0a, 32, net->e0a, P0, 32, net->g0a));
  RCHK_(conv3_bwd(net, s, L_E0A, net->x0, 8, nullptr, 0, net->g0a, B, H, W, nullptr));
  return rc;
}

}  // namespace

namespace wsi {

long long param_count() {
  long long n = 0;
  for (const Spec& s : kSpecs)
    n += (s.kind == CONV3 ? 9LL * s.cin * s.cout : s.kind == TCONV2 ? 4LL * s.cin * s.cout : s.cin) + s.cout;
  return n;
}

void native(const ws_net* net, int* ny, int* nx, int* max_batch) {
  *ny = net->H;
  *nx = net->W;
  *max_batch = net->B;
}

const char* error(const ws_net* net) { return net ? net->err : "no network"; }

int create(ws_net** out, int max_batch, int ny, int nx, char* err, size_t errlen) {
  *out = nullptr;
  if (max_batch < 1 || ny < 8 || nx < 8 || ny % 8 || nx % 8 || ny > 4096 || nx > 4096) {
    std::snprintf(err, errlen, "network size %dx%d (batch %d) unsupported: multiples of 8 up to 4096", ny, nx,
                  max_batch);
    return GP_EUNSUPPORTED;
  }
  if (size_t(max_batch) * size_t(ny) * size_t(nx) >= (size_t(1) << 31)) {  // pixel indices are 32-bit
    std::snprintf(err, errlen, "network batch %d x %dx%d has 2^31 or more pixels", max_batch, ny, nx);
    return GP_EUNSUPPORTED;
  }
  ws_net* n = new (std::nothrow) ws_net();
  if (!n) return GP_ENOMEM;
  n->B = max_batch;
  n->H = ny;
  n->W = nx;
  // parameter blob offsets and packed forms with their gather tables
  std::vector<int> idx;
  size_t o = 0;
  for (int li = 0; li < L_COUNT; ++li) {
    Layer& l = n->L[li];
    l.s = kSpecs[li];
    const int ci = l.s.cin, co = l.s.cout;
    const size_t nw = l.s.kind == CONV3 ? size_t(9) * ci * co : l.s.kind == TCONV2 ? size_t(4) * ci * co : ci;
    l.woff = o;
    l.boff = o + nw;
    o += nw + co;
    auto add = [&](Packed& p, int N, int K, auto src) {
      p.n = N;
      p.npad = rup(N, nt_for(rup(N, 32)));
      p.k = K;
      p.kpad = rup(K, 32);
      p.off = idx.size();
      idx.resize(idx.size() + size_t(p.npad) * p.kpad, -1);
      for (int r = 0; r < N; ++r)
        for (int k = 0; k < K; ++k) idx[p.off + size_t(r) * p.kpad + k] = src(r, k);
    };
    if (l.s.kind == CONV3) {
      const int ct = ci == 2 ? 8 : ci;  // the input layer reads an 8-channel padded tensor
      add(l.fwd, co, 9 * ct, [&](int r, int k) {
        const int tap = k / ct, c = k % ct;
        return c < ci ? int(l.woff + (size_t(r) * 9 + tap) * ci + c) : -1;
      });
      if (li != L_E0A)
        add(l.bwd, ci, 9 * co, [&](int r, int k) {  // [ci][tap'][co] = W[co][8 - tap'][ci]
          const int tap = k / co, c = k % co;
          return int(l.woff + (size_t(c) * 9 + (8 - tap)) * ci + r);
        });
    } else if (l.s.kind == TCONV2) {
      add(l.fwd, 4 * co, ci, [&](int r, int k) {  // [tap co][ci] = Wt[ci][tap][co]
        const int tap = r / co, c = r % co;
        return int(l.woff + (size_t(k) * 4 + tap) * co + c);
      });
      add(l.bwd, ci, 4 * co, [&](int r, int k) { return int(l.woff + size_t(r) * 4 * co + k); });
    }
  }
  n->nparam = o;
  n->npacked = idx.size();
  // activations
  const size_t P0 = size_t(max_batch) * ny * nx, P1 = P0 / 4, P2 = P0 / 16, P3 = P0 / 64;
  struct T {
    bf16** p;
    size_t elems;
  };
  const T ts[] = {{&n->x0, P0 * 8},     {&n->e0a, P0 * 32},   {&n->s0, P0 * 32},    {&n->p0, P1 * 32},
                  {&n->e1a, P1 * 64},   {&n->s1, P1 * 64},    {&n->p1, P2 * 64},    {&n->e2a, P2 * 128},
                  {&n->s2, P2 * 128},   {&n->p2, P3 * 128},   {&n->ma, P3 * 256},   {&n->mb, P3 * 256},
                  {&n->u2, P2 * 128},   {&n->d2a, P2 * 128},  {&n->d2b, P2 * 128},  {&n->u1, P1 * 64},
                  {&n->d1a, P1 * 64},   {&n->d1b, P1 * 64},   {&n->u0, P0 * 32},    {&n->d0a, P0 * 32},
                  {&n->d0b, P0 * 32},   {&n->g0a, P0 * 32},   {&n->g0b, P0 * 32},   {&n->dcat0, P0 * 64},
                  {&n->dd1b, P1 * 64},  {&n->g1a, P1 * 64},   {&n->g1b, P1 * 64},   {&n->dcat1, P1 * 128},
                  {&n->dp0, P1 * 32},   {&n->dd2b, P2 * 128}, {&n->g2a, P2 * 128},  {&n->g2b, P2 * 128},
                  {&n->dcat2, P2 * 256}, {&n->dp1, P2 * 64},  {&n->dmb, P3 * 256},  {&n->g3a, P3 * 256},
                  {&n->g3b, P3 * 256},  {&n->dp2, P3 * 128}};
  size_t bytes = 0;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  for (const T& t : ts) bytes += al(t.elems * sizeof(bf16));
  bytes += 2 * al(P0 * sizeof(float));                          // phi, dphi
  bytes += 4 * al(n->nparam * sizeof(float));                   // par, grad, m1, m2
  bytes += al(n->npacked * sizeof(bf16)) + al(n->npacked * 4);  // packed, gather table
  bytes += al(sizeof(double));
  if (hipMalloc(&n->arena, bytes) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&n->loss_host), sizeof(double)) != hipSuccess) {
    std::snprintf(err, errlen, "network workspace allocation of %zu bytes failed", bytes);
    destroy(n);
    return GP_ENOMEM;
  }
  char* q = static_cast<char*>(n->arena);
  auto take = [&](size_t b) {
    char* r = q;
    q += al(b);
    return r;
  };
  for (const T& t : ts) *t.p = reinterpret_cast<bf16*>(take(t.elems * sizeof(bf16)));
  n->phi = reinterpret_cast<float*>(take(P0 * sizeof(float)));
  n->dphi = reinterpret_cast<float*>(take(P0 * sizeof(float)));
  n->par = reinterpret_cast<float*>(take(n->nparam * sizeof(float)));
  n->grad = reinterpret_cast<float*>(take(n->nparam * sizeof(float)));
  n->m1 = reinterpret_cast<float*>(take(n->nparam * sizeof(float)));
  n->m2 = reinterpret_cast<float*>(take(n->nparam * sizeof(float)));
  n->packed = reinterpret_cast<bf16*>(take(n->npacked * sizeof(bf16)));
  n->pidx = reinterpret_cast<int*>(take(n->npacked * 4));
  n->loss_dev = reinterpret_cast<double*>(take(sizeof(double)));
  bool ok = hipMemcpy(n->pidx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  for (float* b : {n->par, n->grad, n->m1, n->m2}) ok = ok && hipMemset(b, 0, n->nparam * sizeof(float)) == hipSuccess;
  if (!ok) {
    std::snprintf(err, errlen, "network workspace initialisation failed");
    destroy(n);
    return GP_EHIP;
  }
  *out = n;
  return GP_OK;
}

void destroy(ws_net* n) {
  if (!n) return;
  if (n->arena) (void)hipFree(n->arena);
  if (n->loss_host) (void)hipHostFree(n->loss_host);
  delete n;
}

int set_params(ws_net* n, hipStream_t s, const float* blob) {
  WCHK(n, hipMemcpyAsync(n->par, blob, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_fill, dim3(gs(n->nparam)), dim3(256), 0, s, n->m1, n->nparam);
  WLAUNCH(n);
  hipLaunchKernelGGL(k_fill, dim3(gs(n->nparam)), dim3(256), 0, s, n->m2, n->nparam);
  WLAUNCH(n);
  n->t = 0;
  return pack(n, s);
}

int get_params(ws_net* n, hipStream_t s, float* blob) {
  WCHK(n, hipMemcpyAsync(blob, n->par, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  return GP_OK;
}

int predict(ws_net* n, hipStream_t s, const float* r0, const float* r1, int batch, float* phi) {
  if (batch < 1 || batch > n->B) {
    std::snprintf(n->err, sizeof(n->err), "batch %d outside [1, %d]", batch, n->B);
    return GP_EINVAL;
  }
  int rc = forward(n, s, r0, r1, batch);
  if (rc) return rc;
  WCHK(n, hipMemcpyAsync(phi, n->phi, size_t(batch) * n->H * n->W * sizeof(float), hipMemcpyDeviceToDevice, s));
  return GP_OK;
}

int grads(ws_net* n, hipStream_t s, const float* r0, const float* r1, const float* star, int batch, double h,
          float* grad_out, double* loss) {
  if (batch < 1 || batch > n->B || !(h > 0)) {
    std::snprintf(n->err, sizeof(n->err), "batch %d outside [1, %d] or h <= 0", batch, n->B);
    return GP_EINVAL;
  }
  hipLaunchKernelGGL(k_fill, dim3(gs(n->nparam)), dim3(256), 0, s, n->grad, n->nparam);
  WLAUNCH(n);
  hipLaunchKernelGGL(k_fill64, dim3(1), dim3(1), 0, s, n->loss_dev);
  WLAUNCH(n);
  int rc = forward(n, s, r0, r1, batch);
  if (rc) return rc;
  const size_t P0 = size_t(batch) * n->H * n->W;
  hipLaunchKernelGGL(k_loss, dim3(gs(P0) < 1024 ? gs(P0) : 1024), dim3(256), 0, s, n->phi, star, batch, n->H, n->W,
                     1.0 / h, 1.0 / double(P0), n->dphi, n->loss_dev);
  WLAUNCH(n);
  rc = backward(n, s, batch);
  if (rc) return rc;
  if (grad_out) WCHK(n, hipMemcpyAsync(grad_out, n->grad, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  WCHK(n, hipMemcpyAsync(n->loss_host, n->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  WCHK(n, hipStreamSynchronize(s));
  if (loss) *loss = *n->loss_host / double(P0);
  return GP_OK;
}

int adam(ws_net* n, hipStream_t s, double lr) {
  n->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = float(1.0 - std::pow(b1, double(n->t))), c2 = float(1.0 - std::pow(b2, double(n->t)));
  hipLaunchKernelGGL(k_adam, dim3(gs(n->nparam)), dim3(256), 0, s, n->par, n->grad, n->m1, n->m2, n->nparam,
                     float(lr), float(b1), float(b2), float(1.0 - b1), float(1.0 - b2), 1e-8f, c1, c2);
  WLAUNCH(n);
  return pack(n, s);
}

int downsample(hipStream_t s, const float* in, int ny, int nx, int f, float* out) {
  hipLaunchKernelGGL(k_down, dim3(gs(size_t(ny / f) * (nx / f))), dim3(256), 0, s, in, ny, nx, f, out);
  return hipGetLastError() == hipSuccess ? GP_OK : GP_EHIP;
}

int upsample(hipStream_t s, const float* in, int ny, int nx, int f, float* out) {
  hipLaunchKernelGGL(k_up, dim3(gs(size_t(ny) * f * nx * f)), dim3(256), 0, s, in, ny, nx, f, out);
  return hipGetLastError() == hipSuccess ? GP_OK : GP_EHIP;
}

}  // namespace wsi
