// 3-D grid kernels: the d = 3 case of the method of section 3 (the theory of
// sections 2-3 holds for any dimension; the 2-D kernels' discretisation with
// a third axis).
//
// Layout: scalar fields [nz][ny][nx] row-major (x fastest), vector fields
// planar [3][nz][ny][nx] (components x, y, z).  Gradient: forward differences,
// zero on the far faces; divergence: its negative adjoint (backward
// differences).  The screened Poisson solve (alpha I - Delta)^{-1} is a 3-D
// DCT-II in five passes over the field:
//   x forward   k_rows_fwd  (rows of the [nz ny][nx] view, written to the
//                            strip-tiled intermediate of each z-plane); in the
//                            solvers k3_rows_fwd_rhs, which forms the
//                            right-hand side in its loads
//   y forward   k3_cols_dct<.., false> (columns of each z-plane's tiles)
//   z solve     k_cols_solve over the [nz][ny nx] view: DCT-II along z,
//               scale by 1/(nx ny nz (alpha + mu_z + mu_y + mu_x)), inverse
//               (the y, x eigenvalue sum comes from a table laid out like the
//               plane's tiled intermediate)
//   y inverse   k3_cols_dct<.., true>
//   x inverse   k_rows_inv (back to row-major)
#pragma once
#include <hip/hip_runtime.h>

#include "gprox_fft.hpp"
#include "gprox_kernels.hpp"

namespace gp {

// One direction of the y-axis DCT-II over the strip-tiled intermediate of a
// stack of z-planes (blockIdx.y = plane): forward leaves the spectrum in
// natural frequency order along the column, inverse (times N) takes it from
// there.  Column addressing as in k_cols_solve: two adjacent columns per FFT
// group, strips of TW = 2^lgtw columns stored row-major and contiguous.
template <int N, class C, bool INV>
__global__ __launch_bounds__((ColShape<N, C>::MAXTHREADS), (ColShape<N, C>::MINW)) void k3_cols_dct(
    typename Cx<C>::R* buf, int nx, const C* __restrict__ tw, const C* __restrict__ dctw, int lgtw) {
  using Re = typename Cx<C>::R;
  using SH = ColShape<N, C>;
  buf += size_t(blockIdx.y) * N * nx;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int G = blockDim.x / SH::T;
  const int g = threadIdx.x % G, t = threadIdx.x / G;
  C* lds = smem + g * Sched<N>::LDS;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int TW = 1 << lgtw, per = TW / (2 * G);
  const int strip = blk / per, sub = blk - strip * per;
  const int c = strip * TW + 2 * (sub * G + g);
  const bool valid = c < nx;
  Re* col = buf + (valid ? size_t(strip) * N * TW + 2 * (sub * G + g) : 0);
  const int ld = TW;
  Vals<N, C> v;
  if constexpr (!INV) {
    dct2_fwd<N>(t, v, lds, tw, dctw, [&](int m, C& A, C& B) {
      if (valid) {
        const C L0 = *reinterpret_cast<const C*>(col + size_t(2 * m) * ld);
        const C L1 = *reinterpret_cast<const C*>(col + size_t(2 * m + 1) * ld);
        A = mk<C>(L0.x, L1.x);
        B = mk<C>(L0.y, L1.y);
      } else {
        A = mk<C>(Re(0), Re(0));
        B = A;
      }
    });
    if (valid) {
#pragma unroll
      for (int slot = 0; slot < 2; ++slot)
#pragma unroll
        for (int s = 0; s < Sched<N>::H; ++s)
          *reinterpret_cast<C*>(col + size_t(dc_index<N>(t, slot, s)) * ld) = v[slot * Sched<N>::H + s];
    }
  } else {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot)
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s)
        v[slot * Sched<N>::H + s] =
            valid ? *reinterpret_cast<const C*>(col + size_t(dc_index<N>(t, slot, s)) * ld) : mk<C>(Re(0), Re(0));
    dct2_inv<N>(t, v, lds, tw, dctw[t], [&](int m, C A, C B) {
      if (valid) {
        *reinterpret_cast<C*>(col + size_t(2 * m) * ld) = mk<C>(A.x, B.x);
        *reinterpret_cast<C*>(col + size_t(2 * m + 1) * ld) = mk<C>(A.y, B.y);
      }
    });
  }
}

// x-forward DCT-II pass fused with the right-hand side it transforms, formed
// in the loads of the FFT's first pass (Makhoul pairs (2m, 2m+1) of each row
// pair) and never stored:
//   ROF (C = float2):  r = lambda tau (I - u) + tau div pbar
//   EMD (C = double2): b = -div w / h in FP64 (w the stored field)
// V is the planar vector field whose divergence is taken (pbar or w; backward
// differences, far-face components read as zero, every halo load issued
// unconditionally from an in-bounds address and masked); rows of the
// [nz ny][N] view, output to each plane's strip-tiled intermediate as
// k_rows_fwd.  (0 I - Delta) phi = b then gives Delta phi = div w.
template <int N, class C, bool EMD>
__global__ __launch_bounds__((RowShape<N, C>::MAXT), (RowShape<N, C>::MINW)) void k3_rows_fwd_rhs(
    const float* __restrict__ u, const float* __restrict__ V, const float* __restrict__ I,
    typename Cx<C>::R* __restrict__ out, int nz, int ny, int lgtw, float lt, float tau_h, double inv_h,
    const C* __restrict__ tw, const C* __restrict__ dctw) {
  using Re = typename Cx<C>::R;
  using SH = RowShape<N, C>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* smem = reinterpret_cast<C*>(smem_raw);
  const int g = threadIdx.x / SH::T, t = threadIdx.x % SH::T;
  C* lds = smem + g * Sched<N>::LDS;
  const int rows = nz * ny;
  const int ra = 2 * (blockIdx.x * int(blockDim.x / SH::T) + g), rb = ra + 1;
  const bool va = ra < rows;  // rows is even: rb exists with ra
  const size_t n = size_t(rows) * N, P = size_t(ny) * N;
  const float* vx = V;
  const float* vy = V + n;
  const float* vz = V + 2 * n;
  // right-hand side at (row, 2m) and (row, 2m + 1); an out-of-range row pair reads row 0 and is not stored
  auto rhs2 = [&](int row, int m, Re& r0, Re& r1) {
    const int i = row % ny, k = row / ny;
    const bool hy = i < ny - 1, ly = i > 0, hz = k < nz - 1, lz = k > 0, lx0 = m > 0, hx1 = 2 * m + 1 < N - 1;
    const size_t base = size_t(row) * N + 2 * m;
    const float2 X = *reinterpret_cast<const float2*>(vx + base);
    const float Xl = vx[base - (lx0 ? 1 : 0)];
    const float2 Y = *reinterpret_cast<const float2*>(vy + base);
    const float2 Ym = *reinterpret_cast<const float2*>(vy + base - (ly ? size_t(N) : 0));
    const float2 Z = *reinterpret_cast<const float2*>(vz + base);
    const float2 Zm = *reinterpret_cast<const float2*>(vz + base - (lz ? P : 0));
    if constexpr (!EMD) {
      const float2 U = *reinterpret_cast<const float2*>(u + base);
      const float2 J = *reinterpret_cast<const float2*>(I + base);
      float d0 = 0.f, d1 = 0.f;
      d0 += X.x - (lx0 ? Xl : 0.f);
      d0 += (hy ? Y.x : 0.f) - (ly ? Ym.x : 0.f);
      d0 += (hz ? Z.x : 0.f) - (lz ? Zm.x : 0.f);
      d1 += (hx1 ? X.y : 0.f) - X.x;
      d1 += (hy ? Y.y : 0.f) - (ly ? Ym.y : 0.f);
      d1 += (hz ? Z.y : 0.f) - (lz ? Zm.y : 0.f);
      r0 = lt * (J.x - U.x) + tau_h * d0;
      r1 = lt * (J.y - U.y) + tau_h * d1;
    } else {
      double d0 = 0.0, d1 = 0.0;
      d0 += double(X.x) - double(lx0 ? Xl : 0.f);
      d0 += double(hy ? Y.x : 0.f) - double(ly ? Ym.x : 0.f);
      d0 += double(hz ? Z.x : 0.f) - double(lz ? Zm.x : 0.f);
      d1 += double(hx1 ? X.y : 0.f) - double(X.x);
      d1 += double(hy ? Y.y : 0.f) - double(ly ? Ym.y : 0.f);
      d1 += double(hz ? Z.y : 0.f) - double(lz ? Zm.y : 0.f);
      r0 = -d0 * inv_h;
      r1 = -d1 * inv_h;
    }
  };
  const int la = va ? ra : 0, lb = va ? rb : 1;
  Vals<N, C> v;
  dct2_fwd<N>(t, v, lds, tw, dctw, [&](int m, C& A, C& B) {
    Re a0, a1, b0, b1;
    rhs2(la, m, a0, a1);
    rhs2(lb, m, b0, b1);
    A = mk<C>(a0, a1);
    B = mk<C>(b0, b1);
  });
  if (va) {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const SlotTile<N> ta(ra, t, slot, ny, lgtw), tb(rb, t, slot, ny, lgtw);
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s) {
        out[ta.at(s)] = v[slot * Sched<N>::H + s].x;
        out[tb.at(s)] = v[slot * Sched<N>::H + s].y;
      }
    }
  }
}

// Eigenvalue sums mu_y[ky] + mu_x[kx] of one z-plane, laid out like the
// plane's strip-tiled intermediate (the z pass reads them per column).
__global__ __launch_bounds__(256) void k3_mu_plane(const double* __restrict__ muy, const double* __restrict__ mux,
                                                   double* __restrict__ o64, float* __restrict__ o32, int ny, int nx,
                                                   int lgtw) {
  const size_t P = size_t(ny) * nx;
  for (size_t q = size_t(blockIdx.x) * blockDim.x + threadIdx.x; q < P; q += size_t(gridDim.x) * blockDim.x) {
    const size_t TW = size_t(1) << lgtw;
    const size_t strip = q / (size_t(ny) * TW), r = q - strip * size_t(ny) * TW;
    const int ky = int(r / TW), kx = int(strip * TW + (r - size_t(ky) * TW));
    const double v = muy[ky] + mux[kx];
    o64[q] = v;
    o32[q] = float(v);
  }
}

// cell (j, i, k) of a 3-D launch: x over blockIdx.x * blockDim.x + threadIdx.x
// (nx a multiple of blockDim.x), y over blockIdx.y, z over blockIdx.z.
// Neighbour offsets: a neighbour that does not exist is replaced by the cell
// itself, so every halo load is issued unconditionally from an in-bounds
// address and masked afterwards (a load under a branch makes the compiler wait
// for the loads before it); a forward difference with the cell itself is
// exactly zero.
struct Cell3 {
  int j, i, k;
  size_t o;
  bool hx, hy, hz, lx, ly, lz;  // forward / backward neighbour exists along x, y, z
  size_t fx, fy, fz, bx, by, bz;  // offsets to them (0 where they do not exist)
  __device__ __forceinline__ Cell3(int nz, int ny, int nx) {
    j = blockIdx.x * blockDim.x + threadIdx.x;
    i = blockIdx.y;
    k = blockIdx.z;
    o = (size_t(k) * ny + i) * nx + j;
    const size_t P = size_t(ny) * nx;
    hx = j < nx - 1;
    hy = i < ny - 1;
    hz = k < nz - 1;
    lx = j > 0;
    ly = i > 0;
    lz = k > 0;
    fx = hx ? 1 : 0;
    fy = hy ? size_t(nx) : 0;
    fz = hz ? P : 0;
    bx = lx ? 1 : 0;
    by = ly ? size_t(nx) : 0;
    bz = lz ? P : 0;
  }
};

__device__ __forceinline__ void proj_ball3(float& x, float& y, float& z, int aniso) {
  if (aniso) {
    x = fminf(1.f, fmaxf(-1.f, x));
    y = fminf(1.f, fmaxf(-1.f, y));
    z = fminf(1.f, fmaxf(-1.f, z));
  } else {
    const float n2 = x * x + y * y + z * z;
    const float s = n2 > 1.f ? __builtin_amdgcn_rsqf(n2) : 1.f;
    x *= s;
    y *= s;
    z *= s;
  }
}

__device__ __forceinline__ float pnorm3(float x, float y, float z, int aniso) {
  const float n2 = x * x + y * y + z * z;
  return aniso ? fabsf(x) + fabsf(y) + fabsf(z) : (n2 > 0.f ? __builtin_amdgcn_sqrtf(n2) : 0.f);
}

// ---------------------------------------------------------------- ROF (section 3.1 updates)
// u+ = u + delta, then the dual step p+ = proj(p + sigma grad u+), pbar+ = 2 p+ - p
// (u+ at the three forward neighbours formed from their own u and delta).
// u_out must not alias u_in; p and pbar are updated in place.
__global__ __launch_bounds__(256) void k3_rof_update(const float* __restrict__ u_in, const float* __restrict__ d,
                                                     float* __restrict__ p, float* __restrict__ pbar,
                                                     float* __restrict__ u_out, int nz, int ny, int nx, float sig_h,
                                                     int aniso) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const float uc = u_in[c.o] + d[c.o];
  const float ux = u_in[c.o + c.fx] + d[c.o + c.fx], uy = u_in[c.o + c.fy] + d[c.o + c.fy],
              uz = u_in[c.o + c.fz] + d[c.o + c.fz];
  const float gx = c.hx ? ux - uc : 0.f;
  const float gy = c.hy ? uy - uc : 0.f;
  const float gz = c.hz ? uz - uc : 0.f;
  const float ox = p[c.o], oy = p[c.o + n], oz = p[c.o + 2 * n];
  float qx = ox + sig_h * gx, qy = oy + sig_h * gy, qz = oz + sig_h * gz;
  proj_ball3(qx, qy, qz, aniso);
  p[c.o] = qx;
  p[c.o + n] = qy;
  p[c.o + 2 * n] = qz;
  pbar[c.o] = 2.f * qx - ox;
  pbar[c.o + n] = 2.f * qy - oy;
  pbar[c.o + 2 * n] = 2.f * qz - oz;
  u_out[c.o] = uc;
}

// ROF gap partials [sum |grad u|, sum (u - I)^2, sum I div p, sum (div p)^2]
// (differences in grid units); grid-stride over the cells, lgx = log2 nx,
// lgy = log2 ny.
__global__ __launch_bounds__(256) void k3_rof_energy(const float* __restrict__ u, const float* __restrict__ p,
                                                     const float* __restrict__ I, int nz, int ny, int nx, int lgx,
                                                     int lgy, int aniso, double* __restrict__ partials) {
  double acc[4] = {0, 0, 0, 0};
  const size_t n = size_t(nz) * ny * nx, P = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int j = int(o & size_t(nx - 1)), i = int((o >> lgx) & size_t(ny - 1)), k = int(o >> (lgx + lgy));
    const float uc = u[o];
    const float gx = j < nx - 1 ? u[o + 1] - uc : 0.f;
    const float gy = i < ny - 1 ? u[o + nx] - uc : 0.f;
    const float gz = k < nz - 1 ? u[o + P] - uc : 0.f;
    float d = 0.f;
    d += (j < nx - 1 ? p[o] : 0.f) - (j > 0 ? p[o - 1] : 0.f);
    d += (i < ny - 1 ? p[n + o] : 0.f) - (i > 0 ? p[n + o - nx] : 0.f);
    d += (k < nz - 1 ? p[2 * n + o] : 0.f) - (k > 0 ? p[2 * n + o - P] : 0.f);
    const float e = uc - I[o];
    acc[0] += double(pnorm3(gx, gy, gz, aniso));
    acc[1] += double(e) * double(e);
    acc[2] += double(I[o]) * double(d);
    acc[3] += double(d) * double(d);
  }
  const bool mx[4] = {false, false, false, false};
  block_reduce_store<4>(acc, mx, partials);
}

// ---------------------------------------------------------------- EMD (section 3.2 updates, projected form)
// The state between iterations is (w, p) with the stored field w = u - tau pbar
// (u the divergence-free part of the flux): the next projection needs only
// div w (formed in k3_rows_fwd_rhs), and the next update only w at the cell.
// u+ = w - grad phi (the Leray projection of u - tau pbar), p+ = proj(p + sigma
// (u+ + grad psi)), pbar+ = 2 p+ - p, and the next stored field w+ = u+ - tau pbar+.
// Pointwise in w and p (updated in place); phi read at the forward neighbours
// (FP64).  mout (nullable): the flux m = u+ + grad psi [3][n].
__global__ __launch_bounds__(256) void k3_emd_update(float* __restrict__ w, float* __restrict__ p,
                                                     const double* __restrict__ phi, const float* __restrict__ gpsi,
                                                     float* __restrict__ mout, int nz, int ny, int nx, float tau,
                                                     float sigma, double inv_h, int aniso) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const double fc = phi[c.o], fx = phi[c.o + c.fx], fy = phi[c.o + c.fy], fz = phi[c.o + c.fz];
  const float wx = w[c.o], wy = w[n + c.o], wz = w[2 * n + c.o];
  const float ux = c.hx ? wx - float((fx - fc) * inv_h) : 0.f;
  const float uy = c.hy ? wy - float((fy - fc) * inv_h) : 0.f;
  const float uz = c.hz ? wz - float((fz - fc) * inv_h) : 0.f;
  const float mx = ux + gpsi[c.o], my = uy + gpsi[n + c.o], mz = uz + gpsi[2 * n + c.o];
  const float ox = p[c.o], oy = p[n + c.o], oz = p[2 * n + c.o];
  float qx = ox + sigma * mx, qy = oy + sigma * my, qz = oz + sigma * mz;
  proj_ball3(qx, qy, qz, aniso);
  p[c.o] = qx;
  p[n + c.o] = qy;
  p[2 * n + c.o] = qz;
  w[c.o] = ux - tau * (2.f * qx - ox);
  w[n + c.o] = uy - tau * (2.f * qy - oy);
  w[2 * n + c.o] = uz - tau * (2.f * qz - oz);
  if (mout) {
    mout[c.o] = mx;
    mout[n + c.o] = my;
    mout[2 * n + c.o] = mz;
  }
}

// b = -div p / h (FP64): the certificate potential phi_c with Delta phi_c = div p
__global__ __launch_bounds__(256) void k3_div_f64(const float* __restrict__ p, double* __restrict__ b, int nz,
                                                  int ny, int nx, double inv_h) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const float ax = p[c.o], ax0 = p[c.o - c.bx], ay = p[n + c.o], ay0 = p[n + c.o - c.by], az = p[2 * n + c.o],
              az0 = p[2 * n + c.o - c.bz];
  double d = 0.0;
  d += double(c.hx ? ax : 0.f) - double(c.lx ? ax0 : 0.f);
  d += double(c.hy ? ay : 0.f) - double(c.ly ? ay0 : 0.f);
  d += double(c.hz ? az : 0.f) - double(c.lz ? az0 : 0.f);
  b[c.o] = -d * inv_h;
}

// grad psi from the FP64 potential, stored FP32 (planar, 3 components)
__global__ __launch_bounds__(256) void k3_grad_f64(const double* __restrict__ psi, float* __restrict__ g, int nz,
                                                   int ny, int nx, double inv_h) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const double fc = psi[c.o], fx = psi[c.o + c.fx], fy = psi[c.o + c.fy], fz = psi[c.o + c.fz];
  g[c.o] = c.hx ? float((fx - fc) * inv_h) : 0.f;
  g[n + c.o] = c.hy ? float((fy - fc) * inv_h) : 0.f;
  g[2 * n + c.o] = c.hz ? float((fz - fc) * inv_h) : 0.f;
}

// EMD primal partials: sum |m| over the flux m [3][n] (grid-stride over the cells)
__global__ __launch_bounds__(256) void k3_emd_primal(const float* __restrict__ m, size_t n, int aniso,
                                                     double* __restrict__ partials) {
  double acc[1] = {0};
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x)
    acc[0] += double(pnorm3(m[o], m[n + o], m[2 * n + o], aniso));
  const bool mm[1] = {false};
  block_reduce_store<1>(acc, mm, partials);
}

// certificate partials [sum phi f, max |grad phi| (dual norm, 1/h units)]
__global__ __launch_bounds__(256) void k3_emd_cert(const double* __restrict__ phi, const float* __restrict__ f,
                                                   int nz, int ny, int nx, int lgx, int lgy, double inv_h, int aniso,
                                                   double* __restrict__ partials) {
  double acc[2] = {0, 0};
  const size_t n = size_t(nz) * ny * nx, P = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int j = int(o & size_t(nx - 1)), i = int((o >> lgx) & size_t(ny - 1)), k = int(o >> (lgx + lgy));
    const double fc = phi[o];
    const double gx = j < nx - 1 ? (phi[o + 1] - fc) * inv_h : 0.0;
    const double gy = i < ny - 1 ? (phi[o + nx] - fc) * inv_h : 0.0;
    const double gz = k < nz - 1 ? (phi[o + P] - fc) * inv_h : 0.0;
    acc[0] += fc * double(f[o]);
    acc[1] = fmax(acc[1], aniso ? fmax(fmax(fabs(gx), fabs(gy)), fabs(gz)) : gx * gx + gy * gy + gz * gz);
  }
  if (!aniso) acc[1] = sqrt(acc[1]);
  const bool m[2] = {false, true};
  block_reduce_store<2>(acc, m, partials);
}

// ---------------------------------------------------------------- single-variable form (sigma tau = 1)
// With sigma = 1/tau the EMD iteration depends on (u, p, pbar) only through
// y_n = p_{n-1} + sigma (u_n + grad psi), with p_n = proj(y_n) and
// R(y) = 2 proj(y) - y (the Douglas-Rachford case of section 2):
//   phi = Delta^{-1} div R(y_n), u_{n+1} = -tau (R(y_n) - grad phi),
//   y_{n+1} = y_n - proj(y_n) + grad phi + sigma grad psi
// One 3-component field is the whole state; the zero start is y_0 = 0.  (The
// ROF iteration has the same form, but it forms u afresh each iteration, which
// costs FP32 accuracy; ROF keeps the incremental two-variable form.)

// R(y) = 2 proj(y) - y at offset o (all three components: the projection couples them)
__device__ __forceinline__ void refl3(const float* __restrict__ y, size_t n, size_t o, int aniso, float& rx,
                                      float& ry, float& rz) {
  const float yx = y[o], yy = y[n + o], yz = y[2 * n + o];
  float qx = yx, qy = yy, qz = yz;
  proj_ball3(qx, qy, qz, aniso);
  rx = 2.f * qx - yx;
  ry = 2.f * qy - yy;
  rz = 2.f * qz - yz;
}

// EMD: b = -div R(y) / h in FP64: (0 I - Delta) phi = b gives Delta phi = div R(y).
// R couples the three components of y at a cell, so each cell's R is formed
// once and shared: a block is a tile of TX x TY cells of one plane (the x and
// y backward neighbours' R from LDS, the tile's edge threads forming the
// halo's) and marches ZB planes along z, keeping R_z of the previous plane in
// a register.  Launch: block (TX, TY), grid (nx / TX, ny / TY, nz / ZB).
template <int TX, int TY, int ZB>
__global__ __launch_bounds__(TX* TY) void k3_drs_emd_rhs(const float* __restrict__ y, double* __restrict__ b, int nz,
                                                          int ny, int nx, double inv_h, int aniso) {
  __shared__ float sx[TY][TX + 1];  // R_x, column 0: the x halo
  __shared__ float sy[TY + 1][TX];  // R_y, row 0: the y halo
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int j = blockIdx.x * TX + tx, i = blockIdx.y * TY + ty, k0 = blockIdx.z * ZB;
  const size_t n = size_t(nz) * ny * nx, P = size_t(ny) * nx;
  const bool hx = j < nx - 1, lx = j > 0, hy = i < ny - 1, ly = i > 0;
  size_t o = (size_t(k0) * ny + i) * nx + j;
  float Rx, Ry, Rz, t0, t1, rzm = 0.f;
  if (k0 > 0) refl3(y, n, o - P, aniso, t0, t1, rzm);  // R_z of the plane below the first
#pragma unroll 1
  for (int kk = 0; kk < ZB; ++kk) {
    const int k = k0 + kk;
    refl3(y, n, o, aniso, Rx, Ry, Rz);
    sx[ty][tx + 1] = Rx;
    sy[ty + 1][tx] = Ry;
    if (tx == 0) {  // x halo: R_x at j - 1 (the cell itself, masked, at j = 0)
      float hxv, a1, a2;
      refl3(y, n, o - (lx ? 1 : 0), aniso, hxv, a1, a2);
      sx[ty][0] = hxv;
    }
    if (ty == 0) {  // y halo: R_y at i - 1
      float a0, hyv, a2;
      refl3(y, n, o - (ly ? size_t(nx) : 0), aniso, a0, hyv, a2);
      sy[0][tx] = hyv;
    }
    __syncthreads();
    const float Ax = sx[ty][tx], By = sy[ty][tx];
    const bool hz = k < nz - 1, lz = k > 0;
    double d = 0.0;
    d += double(hx ? Rx : 0.f) - double(lx ? Ax : 0.f);
    d += double(hy ? Ry : 0.f) - double(ly ? By : 0.f);
    d += double(hz ? Rz : 0.f) - double(lz ? rzm : 0.f);
    b[o] = -d * inv_h;
    rzm = Rz;
    o += P;
    __syncthreads();  // the next plane overwrites the tile
  }
}

// EMD: y <- y - proj(y) + grad phi + sigma grad psi (in place); mout (nullable):
// the flux of the new iterate, m = u + grad psi = -tau (R(y) - grad phi) + grad psi
__global__ __launch_bounds__(256) void k3_drs_emd_update(float* __restrict__ y, const double* __restrict__ phi,
                                                         const float* __restrict__ gpsi, float* __restrict__ mout,
                                                         int nz, int ny, int nx, float tau, float sigma, double inv_h,
                                                         int aniso) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const double fc = phi[c.o], fx = phi[c.o + c.fx], fy = phi[c.o + c.fy], fz = phi[c.o + c.fz];
  const float gx = c.hx ? float((fx - fc) * inv_h) : 0.f;
  const float gy = c.hy ? float((fy - fc) * inv_h) : 0.f;
  const float gz = c.hz ? float((fz - fc) * inv_h) : 0.f;
  const float yx = y[c.o], yy = y[n + c.o], yz = y[2 * n + c.o];
  const float sx = gpsi[c.o], sy = gpsi[n + c.o], sz = gpsi[2 * n + c.o];
  float qx = yx, qy = yy, qz = yz;
  proj_ball3(qx, qy, qz, aniso);
  y[c.o] = (yx - qx) + gx + sigma * sx;
  y[n + c.o] = (yy - qy) + gy + sigma * sy;
  y[2 * n + c.o] = (yz - qz) + gz + sigma * sz;
  if (mout) {
    mout[c.o] = -tau * ((2.f * qx - yx) - gx) + sx;
    mout[n + c.o] = -tau * ((2.f * qy - yy) - gy) + sy;
    mout[2 * n + c.o] = -tau * ((2.f * qz - yz) - gz) + sz;
  }
}

// warm start of the EMD iteration from a potential phi0: p = proj(grad phi0)
// (forward differences in FP32, zero on the far faces)
__global__ __launch_bounds__(256) void k3_warm_p(const float* __restrict__ phi0, float* __restrict__ p, int nz,
                                                 int ny, int nx, float inv_h, int aniso) {
  const Cell3 c(nz, ny, nx);
  const size_t n = size_t(nz) * ny * nx;
  const float fc = phi0[c.o], fx = phi0[c.o + c.fx], fy = phi0[c.o + c.fy], fz = phi0[c.o + c.fz];
  float qx = c.hx ? (fx - fc) * inv_h : 0.f, qy = c.hy ? (fy - fc) * inv_h : 0.f, qz = c.hz ? (fz - fc) * inv_h : 0.f;
  proj_ball3(qx, qy, qz, aniso);
  p[c.o] = qx;
  p[n + c.o] = qy;
  p[2 * n + c.o] = qz;
}

// p = proj(y), pointwise over n cells (the dual iterate of the single-variable form)
__global__ __launch_bounds__(256) void k3_proj3(const float* __restrict__ y, float* __restrict__ p, size_t n,
                                                int aniso) {
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    float qx = y[o], qy = y[n + o], qz = y[2 * n + o];
    proj_ball3(qx, qy, qz, aniso);
    p[o] = qx;
    p[n + o] = qy;
    p[2 * n + o] = qz;
  }
}

}  // namespace gp
