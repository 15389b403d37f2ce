// HIP kernels for G-prox PDHG on 2-D grids (gfx950).
//
// Discretisation: n_y x n_x cell-centred grid, spacing h, row-major [ny][nx].
//   grad u : forward differences, zero normal component on the far faces;
//   div p  : -grad^T (backward differences);
//   Delta  : div grad, diagonalised by the 2-D DCT-II (appendix A: even
//            reflection turns the Neumann Laplacian into a cosine series);
//   |p|    : collocated Euclidean norm sqrt(px^2 + py^2) (sections 3.1, 3.2).
// Vector fields are planar: component x at [0][ny][nx], y at [1][ny][nx].
#pragma once
#include <hip/hip_runtime.h>

#include "gprox_fft.hpp"

namespace gp {

// ------------------------------------------------------------ launch shapes
// Launch shapes.  The number of FFT groups per block is a launch-time choice
// (blockDim.x / T): the defaults below, or what the library's autotuner
// measured best; the limits keep blocks within 256 threads (row passes, whole
// waves) or 512 threads (column pass), and within the CU's 160 KB of LDS.
template <int N, class C> struct RowShape {
  static constexpr int T = Sched<N>::T;
  static constexpr int MAXT = Sched<N>::E == 16 ? 512 : 256;  // threads per block
  // waves per SIMD the registers must allow: two 512-thread FP32 blocks per CU
  // (their LDS fits); FP64 blocks fill the LDS alone
  static constexpr int MINW = Sched<N>::E == 16 ? (sizeof(C) == 16 ? 2 : 4) : 1;
  static constexpr size_t GROUP_LDS = size_t(Sched<N>::LDS) * sizeof(C);
  static constexpr int G1 = MAXT / T;
  static constexpr int G2 = int(147456 / GROUP_LDS);
  static constexpr int G3 = G1 < G2 ? G1 : G2;
  // whole 64-lane waves (the fused kernels reduce across waves)
  static constexpr int GM = T >= 64 ? 1 : 64 / T;
  static constexpr int G = (G3 / GM) * GM;  // default row pairs per block
  static constexpr int GMAX = G;            // largest allowed
  static constexpr int THREADS = G * T;
  static_assert(G >= 1 && THREADS % 64 == 0 && THREADS <= MAXT, "row-pass shape");
  static constexpr size_t LDS_BYTES = size_t(G) * GROUP_LDS;
};
template <int N, class C> struct ColShape {
  static constexpr int T = Sched<N>::T;
  static constexpr int MAXT = Sched<N>::E == 16 ? 1024 : 512;
  static constexpr size_t GROUP_LDS = size_t(Sched<N>::LDS) * sizeof(C);
  static constexpr int G0 = int(147456 / GROUP_LDS);
  static constexpr int G = G0 > 16 ? 16 : (G0 < 1 ? 1 : G0);  // default column pairs per block
  static constexpr int GL = int(163840 / GROUP_LDS) < MAXT / T ? int(163840 / GROUP_LDS) : MAXT / T;
  static constexpr int GL2 = GL > 64 ? 64 : GL;
  static constexpr int GMAX = GL2 >= 64 ? 64 : GL2 >= 32 ? 32 : GL2 >= 16 ? 16 : GL2 >= 8 ? 8 : GL2 >= 4 ? 4 : GL2 >= 2 ? 2 : 1;
  static constexpr int THREADS = T * G;
  static constexpr int MAXTHREADS = T * (GMAX > G ? GMAX : G);
  static_assert(MAXTHREADS <= 1024, "column-pass shape");
  static constexpr size_t LDS_BYTES = size_t(G) * GROUP_LDS;
  // waves per SIMD the register budget must allow
  static constexpr int MINW0 = MAXTHREADS / 256;
  static constexpr int MINW = Sched<N>::E == 16 ? (MINW0 < 1 ? 1 : MINW0) : (sizeof(C) == 8 ? 2 : 1);
};

// Layout of the row-transformed intermediate (the field between the row and
// column passes): column strips of TW = 2^lgtw columns, each strip stored
// row-major and contiguous, so the column pass streams whole strips and a row
// pass writes TW consecutive values of each of its rows next to each other.
__device__ __forceinline__ size_t tile_idx(int i, int k, int ny, int lgtw) {
  return (size_t(k >> lgtw) * size_t(ny) + size_t(i)) * (size_t(1) << lgtw) + (k & ((1 << lgtw) - 1));
}

// Batches: m instances of one size are stacked into one tall image of m * nyi
// rows (instance-major; vector fields component-major over the whole batch).
// Row a of the tall image is row a % nyi of instance a / nyi; the tiled
// intermediate is tiled per instance.
__device__ __forceinline__ size_t btile(int a, int k, int nyi, int nx, int lgtw) {
  const int inst = a / nyi;
  return size_t(inst) * size_t(nyi) * size_t(nx) + tile_idx(a - inst * nyi, k, nyi, lgtw);
}
__device__ __forceinline__ bool inst_active(const int* active, int inst) { return !active || active[inst] != 0; }

// Offset of spectrum value (slot, s) of row a in the tiled intermediate.  The
// H values of a slot are the indices b + s N/H; when N/H is a multiple of the
// strip width they sit at a constant stride (N/H) nyi from the first one.  For
// N/H >= 128 that holds for every strip width (the settings allow at most 64
// columns, and twice the column-pass groups per block stays below that for
// these lengths); for shorter sequences it is checked per row.
template <int N> struct SlotTile {
  static constexpr int NH = N / Sched<N>::H;
  static constexpr bool ALWAYS = Sched<N>::E == 16 && NH >= 128;
  size_t base;
  int nyi, lgtw, a, b0;
  bool cst;
  __device__ __forceinline__ SlotTile(int a_, int t, int slot, int nyi_, int lgtw_)
      : nyi(nyi_), lgtw(lgtw_), a(a_), b0(0), cst(false) {
    b0 = slot == 0 ? t : ((t == 0) ? N / (2 * Sched<N>::H) : NH - t);
    base = btile(a, b0, nyi, N, lgtw);
    cst = (NH & ((1 << lgtw) - 1)) == 0;
  }
  __device__ __forceinline__ size_t at(int s) const {
    if constexpr (ALWAYS) return base + size_t(s) * (size_t(NH) * nyi);
    else return cst ? base + size_t(s) * (size_t(NH) * nyi) : btile(a, b0 + s * NH, nyi, N, lgtw);
  }
};

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8).
// Renumbering them so that each XCD takes a contiguous range of the work keeps
// neighbouring row groups -- which share halo rows and the cache lines of the
// tiled intermediate -- under one L2.  A permutation of [0, nb) for any nb.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------ DCT passes
// Forward DCT-II along rows, two rows per FFT group.  out may alias in.
template <int N, class C>
__global__ __launch_bounds__((RowShape<N, C>::MAXT), (RowShape<N, C>::MINW)) void k_rows_fwd(const typename Cx<C>::R* in, typename Cx<C>::R* out, int ny,
                                                  int nyi, const int* __restrict__ active, int lgtw,
                                                  const C* __restrict__ tw, const C* __restrict__ dctw) {
  constexpr int ld = N;
  using Re = typename Cx<C>::R;
  using SH = RowShape<N, C>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int g = threadIdx.x / SH::T, t = threadIdx.x % SH::T;
  C* lds = smem + g * Sched<N>::LDS;
  const int ra = 2 * (blockIdx.x * int(blockDim.x / SH::T) + g), rb = ra + 1;
  const bool va = ra < ny && inst_active(active, ra / nyi), vb = va && rb < ny;
  const Re* pa = in + size_t(va ? ra : 0) * ld;
  const Re* pb = in + size_t(vb ? rb : 0) * ld;
  Vals<N, C> v;
  dct2_fwd<N>(t, v, lds, tw, dctw, [&](int m, C& A, C& B) {
    A = va ? *reinterpret_cast<const C*>(pa + 2 * m) : mk<C>(Re(0), Re(0));
    B = vb ? *reinterpret_cast<const C*>(pb + 2 * m) : mk<C>(Re(0), Re(0));
  });
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const SlotTile<N> ta(ra, t, slot, nyi, lgtw), tb(rb, t, slot, nyi, lgtw);
#pragma unroll
    for (int s = 0; s < Sched<N>::H; ++s) {
      if (va) out[ta.at(s)] = v[slot * Sched<N>::H + s].x;
      if (vb) out[tb.at(s)] = v[slot * Sched<N>::H + s].y;
    }
  }
}

// Inverse of the (unnormalised) DCT-II along rows times N.  out may alias in.
template <int N, class C>
__global__ __launch_bounds__((RowShape<N, C>::MAXT), (RowShape<N, C>::MINW)) void k_rows_inv(const typename Cx<C>::R* in, typename Cx<C>::R* out, int ny,
                                                  int nyi, const int* __restrict__ active, int lgtw,
                                                  const C* __restrict__ tw, const C* __restrict__ dctw) {
  constexpr int ld = N;
  using Re = typename Cx<C>::R;
  using SH = RowShape<N, C>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int g = threadIdx.x / SH::T, t = threadIdx.x % SH::T;
  C* lds = smem + g * Sched<N>::LDS;
  const int ra = 2 * (xcd_block(blockIdx.x, gridDim.x) * int(blockDim.x / SH::T) + g), rb = ra + 1;
  const bool va = ra < ny && inst_active(active, ra / nyi), vb = va && rb < ny;
  Vals<N, C> v;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const SlotTile<N> ta(ra, t, slot, nyi, lgtw), tb(rb, t, slot, nyi, lgtw);
#pragma unroll
    for (int s = 0; s < Sched<N>::H; ++s)
      v[slot * Sched<N>::H + s] = mk<C>(va ? in[ta.at(s)] : Re(0), vb ? in[tb.at(s)] : Re(0));
  }
  dct2_inv<N>(t, v, lds, tw, dctw[t], [&](int m, C A, C B) {
    if (va) *reinterpret_cast<C*>(out + size_t(ra) * ld + 2 * m) = A;
    if (vb) *reinterpret_cast<C*>(out + size_t(rb) * ld + 2 * m) = B;
  });
}

// 1/x for the positive, normal spectral denominators of the column pass: the
// hardware reciprocal in FP32 (1 ulp); in FP64 the hardware reciprocal refined
// by two Newton steps r <- r + r (1 - x r) (error within a few ulp, no
// denormal or infinity handling needed here), about half the instructions of
// a correctly rounded division and without its branches
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Column pass of the screened Poisson solve, in place on the row-transformed
// field: DCT-II along y, scale by 1/(nx ny (alpha + mu_y[k] + mu_x[l])) (the
// zero mode is dropped when alpha = 0), inverse DCT-II along y.  Two adjacent
// columns per FFT group; consecutive lanes take consecutive column pairs so
// every row access of a wave covers G*2 contiguous values.
template <int N, class C>
__global__ __launch_bounds__((ColShape<N, C>::MAXTHREADS), (ColShape<N, C>::MINW)) void k_cols_solve(
    typename Cx<C>::R* buf, int nx, const int* __restrict__ active, const C* __restrict__ tw,
    const C* __restrict__ dctw, const typename Cx<C>::R* __restrict__ mux,
    const typename Cx<C>::R* __restrict__ muy, typename Cx<C>::R alpha, typename Cx<C>::R inv_nn, int lgtw) {
  using Re = typename Cx<C>::R;
  using SH = ColShape<N, C>;
  if (!inst_active(active, blockIdx.y)) return;  // whole workgroup: instance retired
  buf += size_t(blockIdx.y) * N * nx;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int G = blockDim.x / SH::T;  // column pairs per block: strip width 2G
  const int g = threadIdx.x % G, t = threadIdx.x / G;
  C* lds = smem + g * Sched<N>::LDS;
  // XCD-aware strip order: strips that share cache lines run under one L2
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  // strips of TW = 2^lgtw columns are contiguous (tile_idx layout); a block
  // takes 2G of them (TW / 2G blocks per strip)
  const int TW = 1 << lgtw, per = TW / (2 * G);
  const int strip = blk / per, sub = blk - strip * per;
  const int c = strip * TW + 2 * (sub * G + g);
  const bool valid = c < nx;
  Re* col = buf + (valid ? size_t(strip) * N * TW + 2 * (sub * G + g) : 0);
  const int ld = TW;
  // FP64 with 16 values per thread: the spectral-scale operands are loaded before
  // the forward transform so that their latency hides behind it (FP32, and FP64
  // with 32 values per thread, keep their registers for the FFT)
  constexpr bool PRE = sizeof(Re) == 8 && Sched<N>::E == 16;
  Re muv[PRE ? 2 * Sched<N>::H : 1];
  Re mxa = Re(0), mxb = Re(0);
  C wti{};  // with PRE: the inverse transform's DCT twiddle base, loaded early as well
  if constexpr (PRE) {
    wti = dctw[t];
#pragma unroll
    for (int slot = 0; slot < 2; ++slot)
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s) muv[slot * Sched<N>::H + s] = muy[dc_index<N>(t, slot, s)];
    if (valid) {
      mxa = mux[c];
      mxb = mux[c + 1];
    }
  }
  Vals<N, C> v;
  dct2_fwd<N>(t, v, lds, tw, dctw, [&](int m, C& A, C& B) {
    if (valid) {
      C L0 = *reinterpret_cast<const C*>(col + size_t(2 * m) * ld);
      C L1 = *reinterpret_cast<const C*>(col + size_t(2 * m + 1) * ld);
      A = mk<C>(L0.x, L1.x);
      B = mk<C>(L0.y, L1.y);
    } else {
      A = mk<C>(Re(0), Re(0));
      B = A;
    }
  });
  if constexpr (!PRE) {
    if (valid) {
      mxa = mux[c];
      mxb = mux[c + 1];
    }
  }
#pragma unroll
  for (int slot = 0; slot < 2; ++slot)
#pragma unroll
    for (int s = 0; s < Sched<N>::H; ++s) {
      const Re my = PRE ? muv[PRE ? slot * Sched<N>::H + s : 0] : muy[dc_index<N>(t, slot, s)];
      const Re da = alpha + my + mxa, db = alpha + my + mxb;
      C& z = v[slot * Sched<N>::H + s];
      z.x = da > Re(0) ? z.x * (inv_nn * recip(da)) : Re(0);
      z.y = db > Re(0) ? z.y * (inv_nn * recip(db)) : Re(0);
    }
  dct2_inv<N>(t, v, lds, tw, PRE ? wti : dctw[t], [&](int m, C A, C B) {
    if (valid) {
      *reinterpret_cast<C*>(col + size_t(2 * m) * ld) = mk<C>(A.x, B.x);
      *reinterpret_cast<C*>(col + size_t(2 * m + 1) * ld) = mk<C>(A.y, B.y);
    }
  });
}

// ------------------------------------------------------------ reductions
// Block-level FP64 reductions over 256 threads (4 waves of 64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// reduces K values per thread; thread 0 writes partials[blockIdx.x * K + i]
template <int K>
__device__ __forceinline__ void block_reduce_store(double (&acc)[K], const bool (&is_max)[K], double* partials) {
  __shared__ double red[4][K];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double r = is_max[i] ? wave_max(acc[i]) : wave_sum(acc[i]);
    if (lane == 0) red[w][i] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double r = red[0][i];
      for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = is_max[i] ? fmax(r, red[q][i]) : r + red[q][i];
      partials[size_t(blockIdx.x) * K + i] = r;
    }
  }
}

// Reduce K values over the T consecutive threads of one FFT group (T a power of
// two, groups aligned to T lanes); the group's thread 0 writes out[0..K).  Must be
// called by every thread of the block (it synchronises when T > 64).
template <int K, int T>
__device__ __forceinline__ void group_reduce_store(double (&acc)[K], double* out, int t) {
  if constexpr (T <= 64) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double r = acc[i];
#pragma unroll
      for (int o = T / 2; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
      if (t == 0 && out) out[i] = r;
    }
  } else {
    constexpr int WPG = T / 64;  // waves per group
    __shared__ double red[8][K];  // blocks of up to 512 threads
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double r = wave_sum(acc[i]);
      if (lane == 0) red[w][i] = r;
    }
    __syncthreads();
    if (t == 0 && out) {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        double r = 0;
        for (int q = 0; q < WPG; ++q) r += red[w + q][i];
        out[i] = r;
      }
    }
    __syncthreads();
  }
}

// Per segment s = blockIdx.x: sum (or max) partials[(s*seg + b)*K + i] over
// b < seg into out[s*K + i]; one block of 256 threads per segment, fixed order.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int seg, int K,
                                                  unsigned max_mask, double* __restrict__ out) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* P = partials + size_t(blockIdx.x) * seg * K;
  for (int i = 0; i < K; ++i) {
    const bool mx = (max_mask >> i) & 1u;
    double a = mx ? -INFINITY : 0.0;
    for (int b = threadIdx.x; b < seg; b += blockDim.x) {
      double x = P[size_t(b) * K + i];
      a = mx ? fmax(a, x) : a + x;
    }
    a = mx ? wave_max(a) : wave_sum(a);
    if (lane == 0) red[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = red[0];
      for (int q = 1; q < 4; ++q) r = mx ? fmax(r, red[q]) : r + red[q];
      out[size_t(blockIdx.x) * K + i] = r;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ helpers
__device__ __forceinline__ void proj_ball(float& qx, float& qy, int aniso) {
  if (aniso) {
    qx = fminf(1.f, fmaxf(-1.f, qx));
    qy = fminf(1.f, fmaxf(-1.f, qy));
  } else {
    // scale by 1/|q| outside the unit disc; the hardware reciprocal square root
    // (1 ulp) replaces a correctly rounded sqrt and divide, which cost about
    // twenty instructions per cell on this path
    const float n2 = qx * qx + qy * qy;
    const float s = n2 > 1.f ? __builtin_amdgcn_rsqf(n2) : 1.f;
    qx *= s;
    qy *= s;
  }
}
__device__ __forceinline__ float pnorm(float x, float y, int aniso) {
  const float n2 = x * x + y * y;
  return aniso ? fabsf(x) + fabsf(y) : (n2 > 0.f ? __builtin_amdgcn_sqrtf(n2) : 0.f);
}

// divergence of a planar vector field at (i, j), far-face components treated as 0
__device__ __forceinline__ float div_at(const float* __restrict__ px, const float* __restrict__ py, int i, int j,
                                        int ny, int nx) {
  const size_t o = size_t(i) * nx + j;
  const float xr = (j < nx - 1) ? px[o] : 0.f;
  const float xl = (j > 0) ? px[o - 1] : 0.f;
  const float yu = (i < ny - 1) ? py[o] : 0.f;
  const float yd = (i > 0) ? py[o - nx] : 0.f;
  return (xr - xl) + (yu - yd);
}

// ------------------------------------------------------------ gap evaluation
// partial sums for the ROF gap: [sum |grad u| (per-h units), sum (u-I)^2,
// sum I div p, sum (div p)^2]; gradients and divergences in 1/h units
__global__ __launch_bounds__(256) void k_rof_energy(const float* __restrict__ u, const float* __restrict__ px,
                                                    const float* __restrict__ py, const float* __restrict__ I,
                                                    int ny, int nx, float inv_h, int aniso,
                                                    double* __restrict__ partials) {
  double acc[4] = {0, 0, 0, 0};
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const float uc = u[o];
    const float gx = (j < nx - 1) ? (u[o + 1] - uc) * inv_h : 0.f;
    const float gy = (i < ny - 1) ? (u[o + nx] - uc) * inv_h : 0.f;
    const float d = div_at(px, py, i, j, ny, nx) * inv_h;
    const float e = uc - I[o];
    acc[0] += double(pnorm(gx, gy, aniso));
    acc[1] += double(e) * double(e);
    acc[2] += double(I[o]) * double(d);
    acc[3] += double(d) * double(d);
  }
  const bool mx[4] = {false, false, false, false};
  block_reduce_store<4>(acc, mx, partials);
}

// r = s div v (s = +-1/h); T = float or double output.  Columns over
// blockIdx.x * blockDim.x + threadIdx.x (nx a multiple of blockDim.x), rows
// over blockIdx.y with stride gridDim.y.
template <class T>
__global__ __launch_bounds__(256) void k_div(const float* __restrict__ vx, const float* __restrict__ vy,
                                             T* __restrict__ r, int ny, int nx, int nyi, float s,
                                             const int* __restrict__ active) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  for (int i = blockIdx.y; i < ny; i += gridDim.y) {
    const int inst = i / nyi, il = i - inst * nyi;
    if (!inst_active(active, inst)) continue;
    const size_t o = size_t(i) * nx + j;
    float vxo = vx[o], vyo = vy[o], vxl = vx[o - (j > 0 ? 1 : 0)], vyd = vy[o - (il > 0 ? nx : 0)];
    // all four loads are in flight before any is masked (keeps the compiler
    // from moving a load under the mask's branch)
    asm volatile("" : "+v"(vxo), "+v"(vyo), "+v"(vxl), "+v"(vyd));
    const float xr = (j < nx - 1) ? vxo : 0.f;
    const float xl = (j > 0) ? vxl : 0.f;
    const float yu = (il < nyi - 1) ? vyo : 0.f;
    const float yd = (il > 0) ? vyd : 0.f;
    r[o] = T((xr - xl) + (yu - yd)) * T(s);
  }
}

// primal value of the state (u, grad psi): sum |u + grad psi|
__global__ __launch_bounds__(256) void k_emd_primal(const float* __restrict__ ux, const float* __restrict__ uy,
                                                    const float* __restrict__ gpx, const float* __restrict__ gpy,
                                                    size_t n, int aniso, double* __restrict__ partials) {
  double acc[1] = {0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x)
    acc[0] += double(pnorm(ux[o] + gpx[o], uy[o] + gpy[o], aniso));
  const bool m[1] = {false};
  block_reduce_store<1>(acc, m, partials);
}

// certificate partials per instance (blockIdx.y): [sum phi f, max |grad phi|]
// (gradient in 1/h units) -> partials[(inst * gridDim.x + blockIdx.x) * 2 + i].
// Rows are strided over the blocks and a row's cells over the threads; nx must
// be a multiple of blockDim.x.  A missing neighbour is read as the cell itself,
// so its difference is exactly 0 and every load is unconditional (loads under a
// branch would serialise the memory round trips); the isotropic maximum is
// taken over |g|^2 and rooted once per thread.
__global__ __launch_bounds__(256) void k_emd_cert(const double* __restrict__ phi, const float* __restrict__ f,
                                                  int nyi, int nx, double inv_h, int aniso,
                                                  double* __restrict__ partials) {
  double acc[2] = {0, 0};
  const size_t base = size_t(blockIdx.y) * nyi * nx;
  const int kn = nx / int(blockDim.x);
  for (int i = blockIdx.x; i < nyi; i += gridDim.x) {
    const double* pr = phi + base + size_t(i) * nx;
    const float* fr_ = f + base + size_t(i) * nx;
    const int dn = i < nyi - 1 ? nx : 0;
#pragma unroll 4
    for (int k = 0; k < kn; ++k) {
      const int j = threadIdx.x + k * int(blockDim.x);
      const double fc = pr[j], fr = pr[j + (j < nx - 1 ? 1 : 0)], fu = pr[j + dn];
      const double gx = (fr - fc) * inv_h, gy = (fu - fc) * inv_h;
      acc[0] += fc * double(fr_[j]);
      acc[1] = fmax(acc[1], aniso ? fmax(fabs(gx), fabs(gy)) : gx * gx + gy * gy);
    }
  }
  if (!aniso) acc[1] = sqrt(acc[1]);
  const bool m[2] = {false, true};
  block_reduce_store<2>(acc, m, partials + size_t(blockIdx.y) * gridDim.x * 2);
}

// certificate of a given FP32 potential phi: [sum phi (rho0 - rho1), max |grad_h phi|]
// (same walk as k_emd_cert; nx a multiple of blockDim.x)
__global__ __launch_bounds__(256) void k_phi_cert(const float* __restrict__ phi, const float* __restrict__ r0,
                                                  const float* __restrict__ r1, int ny, int nx, double inv_h,
                                                  int aniso, double* __restrict__ partials) {
  double acc[2] = {0, 0};
  const int kn = nx / int(blockDim.x);
  for (int i = blockIdx.x; i < ny; i += gridDim.x) {
    const size_t row = size_t(i) * nx;
    const int dn = i < ny - 1 ? nx : 0;
#pragma unroll 4
    for (int k = 0; k < kn; ++k) {
      const size_t o = row + threadIdx.x + size_t(k) * blockDim.x;
      const int j = int(o - row);
      const double fc = phi[o], fr = phi[o + (j < nx - 1 ? 1 : 0)], fu = phi[o + dn];
      const double gx = (fr - fc) * inv_h, gy = (fu - fc) * inv_h;
      acc[0] += fc * (double(r0[o]) - double(r1[o]));
      acc[1] = fmax(acc[1], aniso ? fmax(fabs(gx), fabs(gy)) : gx * gx + gy * gy);
    }
  }
  if (!aniso) acc[1] = sqrt(acc[1]);
  const bool m[2] = {false, true};
  block_reduce_store<2>(acc, m, partials);
}

// out = s * in
template <class T>
__global__ __launch_bounds__(256) void k_scale(const T* __restrict__ in, float* __restrict__ out, size_t n,
                                               double s) {
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x)
    out[o] = float(s * in[o]);
}

// ------------------------------------------------------------ ergodic averages
// Running FP64 sums of the iterates for the averages x^N = (1/N) sum_{n<=N} x_n
// that the convergence theorems of section 2 bound.  The sums are FP64 so that
// the average of N FP32 iterates keeps FP32 accuracy at any N.  n4 = n / 4
// float4 groups (grid sides are powers of two >= 64, so n is a multiple of 4);
// first != 0 starts the sum (s = a) instead of adding.
__global__ __launch_bounds__(256) void k_ergodic_add(const float4* __restrict__ a, double2* __restrict__ s,
                                                     size_t n4, int first) {
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n4; o += size_t(gridDim.x) * blockDim.x) {
    const float4 v = a[o];
    double2 lo = make_double2(v.x, v.y), hi = make_double2(v.z, v.w);
    if (!first) {
      const double2 s0 = s[2 * o], s1 = s[2 * o + 1];
      lo.x += s0.x;
      lo.y += s0.y;
      hi.x += s1.x;
      hi.y += s1.y;
    }
    s[2 * o] = lo;
    s[2 * o + 1] = hi;
  }
}

// EMD: the flux m_n = wt - grad phi of the latest iterate (the field the last
// fused step read and the potential it read, as k_emd_finish forms it, here in
// FP64) into sm [2][ny][nx].  One instance.
__global__ __launch_bounds__(256) void k_emd_ergodic_flux(const float* __restrict__ wt,
                                                          const double* __restrict__ phi, double* __restrict__ sm,
                                                          int ny, int nx, double inv_h, int first) {
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const double fc = phi[o];
    const double mx = (j < nx - 1) ? double(wt[o]) - (phi[o + 1] - fc) * inv_h : 0.0;
    const double my = (i < ny - 1) ? double(wt[o + n]) - (phi[o + nx] - fc) * inv_h : 0.0;
    sm[o] = first ? mx : sm[o] + mx;
    sm[o + n] = first ? my : sm[o + n] + my;
  }
}

// EMD: the averaged flux m^N = inv sm (written FP32 to mout [2][n]) and the
// partial sums of its grid norm |m^N| (primal value h^2 sum |m^N|).
__global__ __launch_bounds__(256) void k_emd_ergodic_primal(const double* __restrict__ sm, double inv, size_t n,
                                                            int aniso, float* __restrict__ mout,
                                                            double* __restrict__ partials) {
  double acc[1] = {0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const float mx = float(inv * sm[o]), my = float(inv * sm[o + n]);
    mout[o] = mx;
    mout[o + n] = my;
    acc[0] += double(pnorm(mx, my, aniso));
  }
  const bool m[1] = {false};
  block_reduce_store<1>(acc, m, partials);
}

// ------------------------------------------------------------ set-up (FP64)
// partials: [sum rho0, sum rho1, count(rho0 < 0 or rho1 < 0 or non-finite)]
__global__ __launch_bounds__(256) void k_mass(const float* __restrict__ r0, const float* __restrict__ r1, size_t n,
                                              double* __restrict__ partials) {
  double acc[3] = {0, 0, 0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const float a = r0[o], b = r1[o];
    acc[0] += double(a);
    acc[1] += double(b);
    if (!(a >= 0.f) || !(b >= 0.f) || !isfinite(a) || !isfinite(b)) acc[2] += 1.0;
  }
  const bool m[3] = {false, false, false};
  block_reduce_store<3>(acc, m, partials);
}

// f = rho1 - rho0 - mean (FP64), written in FP64 (for the set-up solve) and FP32
__global__ __launch_bounds__(256) void k_f64_diff(const float* __restrict__ r0, const float* __restrict__ r1,
                                                  const double* __restrict__ sums, double inv_n, size_t n,
                                                  double* __restrict__ f64, float* __restrict__ f32) {
  const double mean = (sums[1] - sums[0]) * inv_n;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const double v = (double(r1[o]) - double(r0[o])) - mean;
    f64[o] = -v;  // the set-up solve is (0 I - Delta) psi = -f
    f32[o] = float(v);
  }
}

// grad psi from the FP64 potential, stored FP32 (planar)
__global__ __launch_bounds__(256) void k_grad_f64(const double* __restrict__ psi, float* __restrict__ gx,
                                                  float* __restrict__ gy, int ny, int nx, double inv_h) {
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const double c = psi[o];
    gx[o] = (j < nx - 1) ? float((psi[o + 1] - c) * inv_h) : 0.f;
    gy[o] = (i < ny - 1) ? float((psi[o + nx] - c) * inv_h) : 0.f;
  }
}

// ------------------------------------------------------------ step-size rules
// Partial sums for the ROF step rule of section 4.1 and the bound on ||u*||_TV of
// section 3.1: [sum |grad I| (grid norm), sum |grad I|_2^2, sum I], the forward
// differences formed in FP64 from the FP32 image (1/h units).
__global__ __launch_bounds__(256) void k_rule_sums(const float* __restrict__ I, int ny, int nx, double inv_h,
                                                   int aniso, double* __restrict__ partials) {
  double acc[3] = {0, 0, 0};
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const double c = I[o];
    const double gx = (j < nx - 1) ? (double(I[o + 1]) - c) * inv_h : 0.0;
    const double gy = (i < ny - 1) ? (double(I[o + nx]) - c) * inv_h : 0.0;
    const double g2 = gx * gx + gy * gy;
    acc[0] += aniso ? fabs(gx) + fabs(gy) : sqrt(g2);
    acc[1] += g2;
    acc[2] += c;
  }
  const bool m[3] = {false, false, false};
  block_reduce_store<3>(acc, m, partials);
}

// [sum (I - mean)^2] with mean = sums[2] * inv_n (the finalised k_rule_sums)
__global__ __launch_bounds__(256) void k_centered_sq(const float* __restrict__ I, size_t n,
                                                     const double* __restrict__ sums, double inv_n,
                                                     double* __restrict__ partials) {
  const double mean = sums[2] * inv_n;
  double acc[1] = {0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const double e = double(I[o]) - mean;
    acc[0] += e * e;
  }
  const bool m[1] = {false};
  block_reduce_store<1>(acc, m, partials);
}

// count of non-finite values (block partials)
__global__ __launch_bounds__(256) void k_nonfinite(const float* __restrict__ x, size_t n,
                                                   double* __restrict__ partials) {
  double acc[1] = {0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x)
    if (!isfinite(x[o])) acc[0] += 1.0;
  const bool m[1] = {false};
  block_reduce_store<1>(acc, m, partials);
}

}  // namespace gp
