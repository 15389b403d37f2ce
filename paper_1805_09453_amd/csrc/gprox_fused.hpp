// Fused G-prox PDHG iteration kernels (gfx950).
//
// One iteration of Algorithm 2 is split into three launches so that no FFT
// ever needs a neighbouring row:
//
//   A (row pass):  the pointwise dual step of the PREVIOUS iteration together
//                  with the right-hand side of the next u-step, evaluated from
//                  stored fields with a one-row / one-column halo, written to
//                  LDS in Makhoul order and transformed by a row DCT-II;
//                  duality-gap partial sums are fused in.
//   C (column pass): DCT-II -> 1/(alpha + mu) -> inverse DCT-II along y
//                  (k_cols_solve in gprox_kernels.hpp).
//   B (row pass):  row inverse DCT-II fused with the primal update.
//
// ROF (section 3.1 updates, incremental form u+ = u + (lambda tau - Delta)^{-1} r):
//   A: p_n = proj(p_{n-1} + sigma grad u_n), pbar_n = 2 p_n - p_{n-1},
//      r_n = lambda tau (I - u_n) + tau div pbar_n            -> row DCT
//   B: u_{n+1} = u_n + delta                                   (row IDCT)
//   HBM bytes per pixel-iteration: A reads u, p, I (16) and writes p, r (12);
//   C reads and writes r (8); B reads r, u and writes u (12): 48 B.
//
// EMD (section 3.2 updates, projected form u+ = P(u - tau pbar)), with the
// stored field wt = u - tau pbar + grad psi:
//   A: m_{n+1} = wt_n - grad phi_n            (= u_{n+1} + grad psi)
//      p_{n+1} = proj(p_n + sigma m_{n+1}), pbar = 2 p_{n+1} - p_n,
//      wt_{n+1} = m_{n+1} - tau pbar,
//      r = f - div wt_{n+1}   (= -div(u_{n+1} - tau pbar), since div grad psi = f)
//                                                             -> row DCT (FP64)
//   B: phi_{n+1} = Delta^{-1} div(u_{n+1} - tau pbar_{n+1})  (row IDCT, FP64)
//   The potential stays FP64 so that grad phi keeps FP32 accuracy.
#pragma once
#include <hip/hip_runtime.h>

#include "gprox_fft.hpp"
#include "gprox_kernels.hpp"

namespace gp {

// Forward DCT-II of two real sequences already in LDS in Makhoul order
// (lds[lpad(m)] = (a, b)-packed v_m).  Layout of the result as dct2_fwd.
template <int N, class C>
__device__ __forceinline__ void dct2_fwd_lds(int t, Vals<N, C>& v, C* lds, const C* __restrict__ tw,
                                             const C* __restrict__ dctw) {
  using S = Sched<N>;
  constexpr int R0 = S::rad(0), H = S::H;
  const C wt = dctw[t];  // exp(-i pi t / 2N), base of this thread's DCT twiddles
  {
    int bi[S::E / R0];
    bidx_seq<N, R0>(t, bi);
    stockham_pass<N, R0, 1, false, true, true>(v, bi, lds, tw + S::toff(0));
  }
  middle_passes<N, false, 1, S::NP - 1, C>(t, v, lds, tw);
  {
    constexpr int PL = S::NP - 1;
    int bi[2];
    bidx_dc<N, H>(t, bi);
    stockham_pass<N, H, S::ls(PL), false, true, false>(v, bi, lds, tw + S::toff(PL));
  }
  dct_split_fwd<N>(t, v, wt);
}

// store (ra, rb) of column j (natural order) into the Makhoul-ordered LDS sequence
template <int N, class C>
__device__ __forceinline__ void mk_put(C* lds, int j, typename Cx<C>::R ra, typename Cx<C>::R rb) {
  const int m = (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1);
  lds[lpad(m)] = mk<C>(ra, rb);
}

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
__device__ __forceinline__ float f4(const float4& v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }
// Loads of halo cells that may not exist are issued unconditionally from an
// in-bounds address and the value is masked afterwards: a load under a branch
// makes the compiler wait for the loads before it, serialising the memory
// round trips of a row pair.
__device__ __forceinline__ float4 sel4(bool c, float4 v) { return c ? v : make_float4(0.f, 0.f, 0.f, 0.f); }
template <class T> __device__ __forceinline__ T sel(bool c, T v) { return c ? v : T(0); }

// pointwise ROF dual step at one cell: p_new = proj(p + s grad u)
__device__ __forceinline__ void rof_dual_pt(float px, float py, float gx, float gy, float s, int aniso, float& ox,
                                            float& oy) {
  ox = px + s * gx;
  oy = py + s * gy;
  proj_ball(ox, oy, aniso);
}

// ---------------------------------------------------------------- ROF A
// mode 0 (steady): p_in = p_{n-1}; computes p_n (written to p_out) and pbar_n.
// mode 1 (entry):  p_in = pbar_n given by the caller; p_out unused.
// Gap partials (PART, mode 0; partials non-null): [sum|grad u|, sum (u-I)^2,
// sum I div p_n, sum (div p_n)^2] in 1/h units.
template <int N, bool PART>
__global__ __launch_bounds__((RowShape<N, float2>::MAXT), (RowShape<N, float2>::MINW)) void k_rof_A(const float* __restrict__ u, const float* __restrict__ pin,
                                               float* __restrict__ pout, const float* __restrict__ I,
                                               float* __restrict__ rhat, int ny, int nyi, const int* __restrict__ active,
                                               int lgtw, float lt, float tau_h, float sig_h, int aniso, int mode,
                                               double* __restrict__ partials, const float2* __restrict__ tw,
                                               const float2* __restrict__ dctw) {
  using SH = RowShape<N, float2>;
  constexpr int T = SH::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* smem = reinterpret_cast<float2*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  float2* lds = smem + g * Sched<N>::LDS;
  const int a = 2 * (blockIdx.x * int(blockDim.x / T) + g), b = a + 1;
  const bool valid = a < ny && inst_active(active, a / nyi);  // nyi is even
  const size_t n = size_t(ny) * N;
  const float* pinx = pin;
  const float* piny = pin + n;
  double acc[4] = {0, 0, 0, 0};
  if (valid) {
    const bool has_up = (a % nyi) > 0, has_dn = ((a + 2) % nyi) != 0;
    const size_t oa = size_t(a) * N, ob = size_t(b) * N, ou = oa - (has_up ? N : 0), od = ob + (has_dn ? N : 0);
#pragma unroll 2
    for (int k = 0; k < Sched<N>::E / 4; ++k) {
      const int c = 4 * (t + T * k);
      const bool has_l = c > 0, has_r = c + 4 < N;
      const int cl = has_l ? c - 1 : c, cr = has_r ? c + 4 : c;  // in-bounds halo columns
      float ra[4], rb[4];
      if (mode == 0) {
        // u at rows a-1, a, b, b+1 (columns c-1 .. c+4 where needed); without a
        // row below, od = ob and uD = uB (the y-difference at b is masked below)
        const float4 uU = sel4(has_up, ld4(u + ou + c));
        const float4 uA = ld4(u + oa + c), uB = ld4(u + ob + c);
        const float4 uD = ld4(u + od + c);
        const float uU4 = sel(has_up && has_r, u[ou + cr]);
        const float uA4 = sel(has_r, u[oa + cr]), uB4 = sel(has_r, u[ob + cr]);
        const float uAl = sel(has_l, u[oa + cl]), uBl = sel(has_l, u[ob + cl]);
        const float uDl = sel(has_l, u[od + cl]);
        // p_{n-1}
        const float4 pxU = sel4(has_up, ld4(pinx + ou + c));
        const float4 pyU = sel4(has_up, ld4(piny + ou + c));
        const float4 pxA = ld4(pinx + oa + c), pyA = ld4(piny + oa + c);
        const float4 pxB = ld4(pinx + ob + c), pyB = ld4(piny + ob + c);
        const float pxAl = sel(has_l, pinx[oa + cl]), pyAl = sel(has_l, piny[oa + cl]);
        const float pxBl = sel(has_l, pinx[ob + cl]), pyBl = sel(has_l, piny[ob + cl]);
        const float4 IA = ld4(I + oa + c), IB = ld4(I + ob + c);
        // p_n and pbar_n at (a-1, c..c+3), (a, c-1..c+3), (b, c-1..c+3); index e = -1..3
        float nxA[5], nyA[5], nxB[5], nyB[5], byU[4], bxA[5], byA[5], bxB[5], byB[5];
#pragma unroll
        for (int e = -1; e < 4; ++e) {
          const int j = c + e;
          const bool inx = j >= 0;
          // row a
          const float ua = e < 0 ? uAl : f4(uA, e);
          const float uan = e < 3 ? f4(uA, e + 1) : uA4;
          const float ub = e < 0 ? uBl : f4(uB, e);
          const float gxa = (j < N - 1) ? (uan - ua) : 0.f;
          const float gya = ub - ua;  // b = a + 1 < ny always
          const float pxa = e < 0 ? pxAl : f4(pxA, e), pya = e < 0 ? pyAl : f4(pyA, e);
          float ox, oy;
          rof_dual_pt(pxa, pya, gxa, gya, sig_h, aniso, ox, oy);
          nxA[e + 1] = inx ? ox : 0.f;
          nyA[e + 1] = inx ? oy : 0.f;
          bxA[e + 1] = inx ? 2.f * ox - pxa : 0.f;
          byA[e + 1] = inx ? 2.f * oy - pya : 0.f;
          // row b
          const float ubn = e < 3 ? f4(uB, e + 1) : uB4;
          const float ud = e < 0 ? uDl : f4(uD, e);
          const float gxb = (j < N - 1) ? (ubn - ub) : 0.f;
          const float gyb = has_dn ? (ud - ub) : 0.f;
          const float pxb = e < 0 ? pxBl : f4(pxB, e), pyb = e < 0 ? pyBl : f4(pyB, e);
          rof_dual_pt(pxb, pyb, gxb, gyb, sig_h, aniso, ox, oy);
          nxB[e + 1] = inx ? ox : 0.f;
          nyB[e + 1] = inx ? oy : 0.f;
          bxB[e + 1] = inx ? 2.f * ox - pxb : 0.f;
          byB[e + 1] = inx ? 2.f * oy - pyb : 0.f;
          if (e >= 0) {
            // row a-1 (only pbar_y is needed)
            const float uu = f4(uU, e), uun = e < 3 ? f4(uU, e + 1) : uU4;
            const float gxu = (j < N - 1) ? (uun - uu) : 0.f;
            const float gyu = f4(uA, e) - uu;
            rof_dual_pt(f4(pxU, e), f4(pyU, e), gxu, gyu, sig_h, aniso, ox, oy);
            byU[e] = has_up ? 2.f * oy - f4(pyU, e) : 0.f;
            // gap partials of (u_n, p_n) at rows a, b
            if constexpr (PART) {
              acc[0] += double(pnorm(gxa, gya, aniso)) + double(pnorm(gxb, gyb, aniso));
              const float ea = f4(uA, e) - f4(IA, e), eb = f4(uB, e) - f4(IB, e);
              acc[1] += double(ea) * ea + double(eb) * eb;
              const float nyU = has_up ? oy : 0.f;
              const float da = ((j < N - 1 ? nxA[e + 1] : 0.f) - nxA[e]) + (nyA[e + 1] - nyU);
              const float db = ((j < N - 1 ? nxB[e + 1] : 0.f) - nxB[e]) + ((has_dn ? nyB[e + 1] : 0.f) - nyA[e + 1]);
              acc[2] += double(f4(IA, e)) * da + double(f4(IB, e)) * db;
              acc[3] += double(da) * da + double(db) * db;
            }
          }
        }
        // the far faces carry no flux
        if (!has_r) {
          nxA[4] = nxB[4] = bxA[4] = bxB[4] = 0.f;
        }
        if (!has_dn) {
#pragma unroll
          for (int e = 0; e < 5; ++e) nyB[e] = byB[e] = 0.f;
        }
        st4(pout + oa + c, make_float4(nxA[1], nxA[2], nxA[3], nxA[4]));
        st4(pout + n + oa + c, make_float4(nyA[1], nyA[2], nyA[3], nyA[4]));
        st4(pout + ob + c, make_float4(nxB[1], nxB[2], nxB[3], nxB[4]));
        st4(pout + n + ob + c, make_float4(nyB[1], nyB[2], nyB[3], nyB[4]));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dva = (bxA[e + 1] - bxA[e]) + (byA[e + 1] - byU[e]);
          const float dvb = (bxB[e + 1] - bxB[e]) + (byB[e + 1] - byA[e + 1]);
          ra[e] = lt * (f4(IA, e) - f4(uA, e)) + tau_h * dva;
          rb[e] = lt * (f4(IB, e) - f4(uB, e)) + tau_h * dvb;
        }
      } else {
        // entry: pbar given
        const float4 uA = ld4(u + oa + c), uB = ld4(u + ob + c);
        const float4 IA = ld4(I + oa + c), IB = ld4(I + ob + c);
        const float4 xA = ld4(pinx + oa + c), yA = ld4(piny + oa + c);
        const float4 xB = ld4(pinx + ob + c), yB = ld4(piny + ob + c);
        const float4 yU = sel4(has_up, ld4(piny + ou + c));
        const float xAl = sel(has_l, pinx[oa + cl]), xBl = sel(has_l, pinx[ob + cl]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = c + e;
          const float xa = (j < N - 1) ? f4(xA, e) : 0.f, xb = (j < N - 1) ? f4(xB, e) : 0.f;
          const float xal = e == 0 ? xAl : f4(xA, e - 1), xbl = e == 0 ? xBl : f4(xB, e - 1);
          const float ya = f4(yA, e), yb = has_dn ? f4(yB, e) : 0.f;
          const float dva = (xa - xal) + (ya - f4(yU, e));
          const float dvb = (xb - xbl) + (yb - ya);
          ra[e] = lt * (f4(IA, e) - f4(uA, e)) + tau_h * dva;
          rb[e] = lt * (f4(IB, e) - f4(uB, e)) + tau_h * dvb;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) mk_put<N, float2>(lds, c + e, ra[e], rb[e]);
    }
  } else {
    // keep the FFT well defined for an idle group (its results are discarded)
#pragma unroll 1
    for (int m = t; m < N; m += T) lds[lpad(m)] = make_float2(0.f, 0.f);
  }
  // gap partials per row pair (so that each instance of a batch has its own)
  if constexpr (PART) group_reduce_store<4, T>(acc, valid ? partials + size_t(a / 2) * 4 : nullptr, t);
  __syncthreads();
  Vals<N, float2> v;
  dct2_fwd_lds<N>(t, v, lds, tw, dctw);
  if (valid) {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const SlotTile<N> ta(a, t, slot, nyi, lgtw), tb(b, t, slot, nyi, lgtw);
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s) {
        rhat[ta.at(s)] = v[slot * Sched<N>::H + s].x;
        rhat[tb.at(s)] = v[slot * Sched<N>::H + s].y;
      }
    }
  }
}

// ---------------------------------------------------------------- ROF B
// u += inverse row DCT of the column-solved field
template <int N>
__global__ __launch_bounds__((RowShape<N, float2>::MAXT), (RowShape<N, float2>::MINW)) void k_rof_B(const float* __restrict__ dhat, float* __restrict__ u, int ny,
                                               int nyi, const int* __restrict__ active, int lgtw,
                                               const float2* __restrict__ tw, const float2* __restrict__ dctw) {
  using SH = RowShape<N, float2>;
  using IO = InvOut<N>;
  constexpr int T = SH::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* smem = reinterpret_cast<float2*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  float2* lds = smem + g * Sched<N>::LDS;
  const int a = 2 * (xcd_block(blockIdx.x, gridDim.x) * int(blockDim.x / T) + g), b = a + 1;
  const bool valid = a < ny && inst_active(active, a / nyi);
  float* ua = u + size_t(valid ? a : 0) * N;
  float* ub = u + size_t(valid ? b : 0) * N;
  Vals<N, float2> v;
#pragma unroll
  for (int slot = 0; slot < 2; ++slot) {
    const SlotTile<N> ta(a, t, slot, nyi, lgtw), tb(b, t, slot, nyi, lgtw);
#pragma unroll
    for (int s = 0; s < Sched<N>::H; ++s)
      v[slot * Sched<N>::H + s] = valid ? make_float2(dhat[ta.at(s)], dhat[tb.at(s)]) : make_float2(0, 0);
  }
  // u at this thread's output positions, loaded before the last pass so the
  // latency overlaps it
  float2 oa[IO::NQ][2][IO::NS], ob[IO::NQ][2][IO::NS];
  dct2_inv_core<N>(t, v, lds, tw, dctw[t], [&] {
#pragma unroll
    for (int q = 0; q < IO::NQ; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < IO::NS; ++s) {
          const int m = IO::m(t, q, h, s);
          oa[q][h][s] = *reinterpret_cast<const float2*>(ua + 2 * m);
          ob[q][h][s] = *reinterpret_cast<const float2*>(ub + 2 * m);
        }
  });
  if (valid) {
#pragma unroll
    for (int q = 0; q < IO::NQ; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < IO::NS; ++s) {
          const int m = IO::m(t, q, h, s);
          float2 x0, x1;
          IO::get(v, q, h, s, x0, x1);
          *reinterpret_cast<float2*>(ua + 2 * m) = make_float2(oa[q][h][s].x + x0.x, oa[q][h][s].y + x1.x);
          *reinterpret_cast<float2*>(ub + 2 * m) = make_float2(ob[q][h][s].x + x0.y, ob[q][h][s].y + x1.y);
        }
  }
}

// ---------------------------------------------------------------- ROF finish
// p_out = proj(p_in + sigma grad u), pbar_out = 2 p_out - p_in (pointwise in p:
// p_in may alias p_out or pbar_out)
__global__ __launch_bounds__(256) void k_rof_finish(const float* __restrict__ u, const float* pin, float* pout,
                                                    float* pbar, int ny, int nx, int nyi, float sig_h, int aniso) {
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const float uc = u[o];
    const float gx = (j < nx - 1) ? (u[o + 1] - uc) : 0.f;
    const float gy = (i % nyi < nyi - 1) ? (u[o + nx] - uc) : 0.f;
    const float ox = pin[o], oy = pin[o + n];
    float qx, qy;
    rof_dual_pt(ox, oy, gx, gy, sig_h, aniso, qx, qy);
    pout[o] = qx;
    pout[o + n] = qy;
    pbar[o] = 2.f * qx - ox;
    pbar[o + n] = 2.f * qy - oy;
  }
}

// ---------------------------------------------------------------- EMD A (FP64 transform)
// mode 0 (steady): wt_in = wt_n, phi = phi_n, p_in = p_n -> p_out = p_{n+1}, wt_out = wt_{n+1};
//                  partials (nullable): [sum |m_{n+1}|].
// mode 1 (entry):  u = u_n (in wt_in's place), p_in = pbar_n, gpsi = grad psi -> wt_out = wt_n.
template <int N, bool PART>
__global__ __launch_bounds__((RowShape<N, double2>::MAXT), (RowShape<N, double2>::MINW)) void k_emd_A(const float* __restrict__ wt_in, const double* __restrict__ phi,
                                               const float* __restrict__ pin, const float* __restrict__ gpsi,
                                               const float* __restrict__ f, float* __restrict__ pout,
                                               float* __restrict__ wt_out, double* __restrict__ rhat, int ny,
                                               int nyi, const int* __restrict__ active, int lgtw, double inv_h,
                                               float tau, float sigma, int aniso, int mode,
                                               double* __restrict__ partials, const double2* __restrict__ tw,
                                               const double2* __restrict__ dctw) {
  using SH = RowShape<N, double2>;
  constexpr int T = SH::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* smem = reinterpret_cast<double2*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  double2* lds = smem + g * Sched<N>::LDS;
  const int a = 2 * (blockIdx.x * int(blockDim.x / T) + g), b = a + 1;
  const bool valid = a < ny && inst_active(active, a / nyi);
  const size_t n = size_t(ny) * N;
  double acc[1] = {0};
  if (valid) {
    const bool has_up = (a % nyi) > 0, has_dn = ((a + 2) % nyi) != 0;
    const size_t oa = size_t(a) * N, ob = size_t(b) * N, ou = oa - (has_up ? N : 0), od = ob + (has_dn ? N : 0);
#pragma unroll 2
    for (int k = 0; k < Sched<N>::E / 4; ++k) {
      const int c = 4 * (t + T * k);
      const bool has_l = c > 0, has_r = c + 4 < N;
      const int cl = has_l ? c - 1 : c, cr = has_r ? c + 4 : c;  // in-bounds halo columns
      // new wt at (a-1, c..c+3) [y only], (a, c-1..c+3), (b, c-1..c+3)
      float wxA[5], wyA[5], wxB[5], wyB[5], wyU[4];
      if (mode == 0) {
        // phi_n rows a-1..b+1
        double fA[6], fB[6], fU[5], fD[5];  // index e+1 for columns c-1..c+4 (fU, fD: c..c+4 / c-1..c+3)
        {
          const double2* pa = reinterpret_cast<const double2*>(phi + oa + c);
          const double2* pb = reinterpret_cast<const double2*>(phi + ob + c);
          double2 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
          fA[1] = a0.x; fA[2] = a0.y; fA[3] = a1.x; fA[4] = a1.y;
          fB[1] = b0.x; fB[2] = b0.y; fB[3] = b1.x; fB[4] = b1.y;
          fA[0] = sel(has_l, phi[oa + cl]);
          fB[0] = sel(has_l, phi[ob + cl]);
          fA[5] = sel(has_r, phi[oa + cr]);
          fB[5] = sel(has_r, phi[ob + cr]);
          // rows a-1 and b+1 (ou = oa, od = ob where they do not exist)
          const double2* pu = reinterpret_cast<const double2*>(phi + ou + c);
          const double2* pd = reinterpret_cast<const double2*>(phi + od + c);
          const double2 u0 = pu[0], u1 = pu[1], d0 = pd[0], d1 = pd[1];
          const double fu4 = phi[ou + cr], fdl = phi[od + cl];
          fU[0] = sel(has_up, u0.x); fU[1] = sel(has_up, u0.y); fU[2] = sel(has_up, u1.x); fU[3] = sel(has_up, u1.y);
          fU[4] = sel(has_up && has_r, fu4);
          fD[1] = sel(has_dn, d0.x); fD[2] = sel(has_dn, d0.y); fD[3] = sel(has_dn, d1.x); fD[4] = sel(has_dn, d1.y);
          fD[0] = sel(has_dn && has_l, fdl);
        }
        const float4 wxa = ld4(wt_in + oa + c), wya = ld4(wt_in + n + oa + c);
        const float4 wxb = ld4(wt_in + ob + c), wyb = ld4(wt_in + n + ob + c);
        const float4 wyu = sel4(has_up, ld4(wt_in + n + ou + c));
        const float4 wxu = sel4(has_up, ld4(wt_in + ou + c));
        const float wxal = sel(has_l, wt_in[oa + cl]), wyal = sel(has_l, wt_in[n + oa + cl]);
        const float wxbl = sel(has_l, wt_in[ob + cl]), wybl = sel(has_l, wt_in[n + ob + cl]);
        const float4 pxa = ld4(pin + oa + c), pya = ld4(pin + n + oa + c);
        const float4 pxb = ld4(pin + ob + c), pyb = ld4(pin + n + ob + c);
        const float4 pxu = sel4(has_up, ld4(pin + ou + c));
        const float4 pyu = sel4(has_up, ld4(pin + n + ou + c));
        const float pxal = sel(has_l, pin[oa + cl]), pyal = sel(has_l, pin[n + oa + cl]);
        const float pxbl = sel(has_l, pin[ob + cl]), pybl = sel(has_l, pin[n + ob + cl]);
        float nxA[4], nyA[4], nxB[4], nyB[4];
#pragma unroll
        for (int e = -1; e < 4; ++e) {
          const int j = c + e;
          const bool inx = j >= 0, xin = j < N - 1;
          // m = wt - grad phi at rows a and b
          const float mxa = xin ? (e < 0 ? wxal : f4(wxa, e)) - float((fA[e + 2] - fA[e + 1]) * inv_h) : 0.f;
          const float mya = (e < 0 ? wyal : f4(wya, e)) - float((fB[e + 1] - fA[e + 1]) * inv_h);
          const float mxb = xin ? (e < 0 ? wxbl : f4(wxb, e)) - float((fB[e + 2] - fB[e + 1]) * inv_h) : 0.f;
          const float myb = has_dn ? (e < 0 ? wybl : f4(wyb, e)) - float((fD[e + 1] - fB[e + 1]) * inv_h) : 0.f;
          const float oxa = e < 0 ? pxal : f4(pxa, e), oya = e < 0 ? pyal : f4(pya, e);
          const float oxb = e < 0 ? pxbl : f4(pxb, e), oyb = e < 0 ? pybl : f4(pyb, e);
          float qxa = oxa + sigma * mxa, qya = oya + sigma * mya;
          float qxb = oxb + sigma * mxb, qyb = oyb + sigma * myb;
          proj_ball(qxa, qya, aniso);
          proj_ball(qxb, qyb, aniso);
          const float bxa = 2.f * qxa - oxa, bya = 2.f * qya - oya;
          const float bxb = 2.f * qxb - oxb, byb = 2.f * qyb - oyb;
          wxA[e + 1] = inx && xin ? mxa - tau * bxa : 0.f;
          wyA[e + 1] = inx ? mya - tau * bya : 0.f;
          wxB[e + 1] = inx && xin ? mxb - tau * bxb : 0.f;
          wyB[e + 1] = inx && has_dn ? myb - tau * byb : 0.f;
          if (e >= 0) {
            nxA[e] = xin ? qxa : 0.f;
            nyA[e] = qya;
            nxB[e] = xin ? qxb : 0.f;
            nyB[e] = has_dn ? qyb : 0.f;
            if constexpr (PART) acc[0] += double(pnorm(mxa, mya, aniso)) + double(pnorm(mxb, myb, aniso));
            // row a-1: y component of the new wt
            if (has_up) {
              const float mxu = xin ? f4(wxu, e) - float((fU[e + 1] - fU[e]) * inv_h) : 0.f;
              const float myu = f4(wyu, e) - float((fA[e + 1] - fU[e]) * inv_h);
              float qxu = f4(pxu, e) + sigma * mxu, qyu = f4(pyu, e) + sigma * myu;
              proj_ball(qxu, qyu, aniso);
              wyU[e] = myu - tau * (2.f * qyu - f4(pyu, e));
            } else {
              wyU[e] = 0.f;
            }
          }
        }
        st4(pout + oa + c, make_float4(nxA[0], nxA[1], nxA[2], nxA[3]));
        st4(pout + n + oa + c, make_float4(nyA[0], nyA[1], nyA[2], nyA[3]));
        st4(pout + ob + c, make_float4(nxB[0], nxB[1], nxB[2], nxB[3]));
        st4(pout + n + ob + c, make_float4(nyB[0], nyB[1], nyB[2], nyB[3]));
      } else {
        // entry: wt_n = u_n - tau pbar_n + grad psi
        const float* ux = wt_in;
        const float* uy = wt_in + n;
#pragma unroll
        for (int e = -1; e < 4; ++e) {
          const int j = c + e;
          const bool inx = j >= 0, xin = j < N - 1;
          const size_t ja = oa + (inx ? j : 0), jb = ob + (inx ? j : 0);
          wxA[e + 1] = inx && xin ? ux[ja] - tau * pin[ja] + gpsi[ja] : 0.f;
          wyA[e + 1] = inx ? uy[ja] - tau * pin[n + ja] + gpsi[n + ja] : 0.f;
          wxB[e + 1] = inx && xin ? ux[jb] - tau * pin[jb] + gpsi[jb] : 0.f;
          wyB[e + 1] = inx && has_dn ? uy[jb] - tau * pin[n + jb] + gpsi[n + jb] : 0.f;
          if (e >= 0) {
            const size_t ju = ou + j;
            wyU[e] = has_up ? uy[ju] - tau * pin[n + ju] + gpsi[n + ju] : 0.f;
          }
        }
      }
      st4(wt_out + oa + c, make_float4(wxA[1], wxA[2], wxA[3], wxA[4]));
      st4(wt_out + n + oa + c, make_float4(wyA[1], wyA[2], wyA[3], wyA[4]));
      st4(wt_out + ob + c, make_float4(wxB[1], wxB[2], wxB[3], wxB[4]));
      st4(wt_out + n + ob + c, make_float4(wyB[1], wyB[2], wyB[3], wyB[4]));
      const float4 FA = ld4(f + oa + c), FB = ld4(f + ob + c);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float dva = (wxA[e + 1] - wxA[e]) + (wyA[e + 1] - wyU[e]);
        const float dvb = (wxB[e + 1] - wxB[e]) + (wyB[e + 1] - wyA[e + 1]);
        mk_put<N, double2>(lds, c + e, double(f4(FA, e)) - double(dva) * inv_h,
                           double(f4(FB, e)) - double(dvb) * inv_h);
      }
    }
  } else {
#pragma unroll 1
    for (int m = t; m < N; m += T) lds[lpad(m)] = make_double2(0.0, 0.0);
  }
  if constexpr (PART) group_reduce_store<1, T>(acc, valid ? partials + size_t(a / 2) : nullptr, t);
  __syncthreads();
  Vals<N, double2> v;
  dct2_fwd_lds<N>(t, v, lds, tw, dctw);
  if (valid) {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const SlotTile<N> ta(a, t, slot, nyi, lgtw), tb(b, t, slot, nyi, lgtw);
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s) {
        rhat[ta.at(s)] = v[slot * Sched<N>::H + s].x;
        rhat[tb.at(s)] = v[slot * Sched<N>::H + s].y;
      }
    }
  }
}

// ---------------------------------------------------------------- EMD A, single-variable form
// With sigma = 1/tau the EMD iterates depend on (u, p, pbar) only through the
// one field y_n = p_{n-1} + sigma (u_n + grad psi) (p_n = proj(y_n); the
// Douglas-Rachford case of section 2); with R(y) = 2 proj(y) - y:
//   phi_n = Delta^{-1} div R(y_n),  u_{n+1} = -tau (R(y_n) - grad phi_n),
//   y_{n+1} = y_n - proj(y_n) + grad phi_n + sigma grad psi.
// mode 0 (steady): y_in = y_n, phi = phi_n -> y_out = y_{n+1}; partials
//                  (nullable): [sum |m_{n+1}|], m = u + grad psi;
// mode 1 (entry):  y_in = y_n -> y_out = y_n.
// Then r = -div R(y_out) / h (FP64) -> row DCT, as k_emd_A.  Reads y, phi and
// grad psi, writes y and the transform: no p, pbar or stored field.
template <int N, bool PART>
__global__ __launch_bounds__((RowShape<N, double2>::MAXT), (RowShape<N, double2>::MINW)) void k_emd_A_drs(
    const float* __restrict__ y_in, const double* __restrict__ phi, const float* __restrict__ gpsi,
    float* __restrict__ y_out, double* __restrict__ rhat, int ny, int nyi, const int* __restrict__ active, int lgtw,
    double inv_h, float tau, float sigma, int aniso, int mode, double* __restrict__ partials,
    const double2* __restrict__ tw, const double2* __restrict__ dctw) {
  using SH = RowShape<N, double2>;
  constexpr int T = SH::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* smem = reinterpret_cast<double2*>(smem_raw);
  const int g = threadIdx.x / T, t = threadIdx.x % T;
  double2* lds = smem + g * Sched<N>::LDS;
  const int a = 2 * (blockIdx.x * int(blockDim.x / T) + g), b = a + 1;
  const bool valid = a < ny && inst_active(active, a / nyi);
  const size_t n = size_t(ny) * N;
  double acc[1] = {0};
  if (valid) {
    const bool has_up = (a % nyi) > 0, has_dn = ((a + 2) % nyi) != 0;
    const size_t oa = size_t(a) * N, ob = size_t(b) * N, ou = oa - (has_up ? N : 0), od = ob + (has_dn ? N : 0);
#pragma unroll 2
    for (int k = 0; k < Sched<N>::E / 4; ++k) {
      const int c = 4 * (t + T * k);
      const bool has_l = c > 0, has_r = c + 4 < N;
      const int cl = has_l ? c - 1 : c, cr = has_r ? c + 4 : c;  // in-bounds halo columns
      // R of the new y at (a, c-1..c+3), (b, c-1..c+3) and, y component only, (a-1, c..c+3)
      float RxA[5], RyA[5], RxB[5], RyB[5], RyU[4];
      float YxA[4], YyA[4], YxB[4], YyB[4];  // the new y at (a, c..c+3), (b, c..c+3)
      const float4 yxa = ld4(y_in + oa + c), yya = ld4(y_in + n + oa + c);
      const float4 yxb = ld4(y_in + ob + c), yyb = ld4(y_in + n + ob + c);
      const float4 yxu = sel4(has_up, ld4(y_in + ou + c)), yyu = sel4(has_up, ld4(y_in + n + ou + c));
      const float yxal = sel(has_l, y_in[oa + cl]), yyal = sel(has_l, y_in[n + oa + cl]);
      const float yxbl = sel(has_l, y_in[ob + cl]), yybl = sel(has_l, y_in[n + ob + cl]);
      // steady mode: grad phi_n and grad psi at the same cells (entry mode: zero step)
      double fA[6] = {0, 0, 0, 0, 0, 0}, fB[6] = {0, 0, 0, 0, 0, 0}, fU[5] = {0, 0, 0, 0, 0}, fD[5] = {0, 0, 0, 0, 0};
      float4 sxa = make_float4(0.f, 0.f, 0.f, 0.f), sya = sxa, sxb = sxa, syb = sxa, sxu = sxa, syu = sxa;
      float sxal = 0.f, syal = 0.f, sxbl = 0.f, sybl = 0.f;
      const bool steady = mode == 0;
      if (steady) {
        const double2* pa = reinterpret_cast<const double2*>(phi + oa + c);
        const double2* pb = reinterpret_cast<const double2*>(phi + ob + c);
        const double2 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
        fA[1] = a0.x; fA[2] = a0.y; fA[3] = a1.x; fA[4] = a1.y;
        fB[1] = b0.x; fB[2] = b0.y; fB[3] = b1.x; fB[4] = b1.y;
        fA[0] = sel(has_l, phi[oa + cl]);
        fB[0] = sel(has_l, phi[ob + cl]);
        fA[5] = sel(has_r, phi[oa + cr]);
        fB[5] = sel(has_r, phi[ob + cr]);
        const double2* pu = reinterpret_cast<const double2*>(phi + ou + c);
        const double2* pd = reinterpret_cast<const double2*>(phi + od + c);
        const double2 u0 = pu[0], u1 = pu[1], d0 = pd[0], d1 = pd[1];
        const double fu4 = phi[ou + cr], fdl = phi[od + cl];
        fU[0] = sel(has_up, u0.x); fU[1] = sel(has_up, u0.y); fU[2] = sel(has_up, u1.x); fU[3] = sel(has_up, u1.y);
        fU[4] = sel(has_up && has_r, fu4);
        fD[1] = sel(has_dn, d0.x); fD[2] = sel(has_dn, d0.y); fD[3] = sel(has_dn, d1.x); fD[4] = sel(has_dn, d1.y);
        fD[0] = sel(has_dn && has_l, fdl);
        sxa = ld4(gpsi + oa + c); sya = ld4(gpsi + n + oa + c);
        sxb = ld4(gpsi + ob + c); syb = ld4(gpsi + n + ob + c);
        sxu = sel4(has_up, ld4(gpsi + ou + c)); syu = sel4(has_up, ld4(gpsi + n + ou + c));
        sxal = sel(has_l, gpsi[oa + cl]); syal = sel(has_l, gpsi[n + oa + cl]);
        sxbl = sel(has_l, gpsi[ob + cl]); sybl = sel(has_l, gpsi[n + ob + cl]);
      }
      // one cell: the new y (steady: y - proj(y) + g + sigma s; entry: y) and its R;
      // (mx, my): the flux of the new iterate (steady mode)
      auto cell = [&](float yx, float yy, float gx, float gy, float sx, float sy, bool hx, bool hy, float& nyx,
                      float& nyy, float& rx, float& ry, float& mx, float& my) {
        float qx = yx, qy = yy;
        proj_ball(qx, qy, aniso);
        if (steady) {
          nyx = hx ? (yx - qx) + gx + sigma * sx : 0.f;
          nyy = hy ? (yy - qy) + gy + sigma * sy : 0.f;
          mx = hx ? -tau * ((2.f * qx - yx) - gx) + sx : 0.f;
          my = hy ? -tau * ((2.f * qy - yy) - gy) + sy : 0.f;
        } else {
          nyx = hx ? yx : 0.f;
          nyy = hy ? yy : 0.f;
          mx = my = 0.f;
        }
        float px = nyx, py = nyy;
        proj_ball(px, py, aniso);
        rx = 2.f * px - nyx;
        ry = 2.f * py - nyy;
      };
#pragma unroll
      for (int e = -1; e < 4; ++e) {
        const int j = c + e;
        const bool inx = j >= 0, xin = j < N - 1;
        float nx0, ny0, rx, ry, mx, my;
        // row a (its row below, b, always exists)
        cell(e < 0 ? yxal : f4(yxa, e), e < 0 ? yyal : f4(yya, e),
             xin ? float((fA[e + 2] - fA[e + 1]) * inv_h) : 0.f, float((fB[e + 1] - fA[e + 1]) * inv_h),
             e < 0 ? sxal : f4(sxa, e), e < 0 ? syal : f4(sya, e), xin, true, nx0, ny0, rx, ry, mx, my);
        RxA[e + 1] = inx ? rx : 0.f;
        RyA[e + 1] = inx ? ry : 0.f;
        if (e >= 0) {
          YxA[e] = nx0;
          YyA[e] = ny0;
          if constexpr (PART) acc[0] += double(pnorm(mx, my, aniso));
        }
        // row b
        cell(e < 0 ? yxbl : f4(yxb, e), e < 0 ? yybl : f4(yyb, e),
             xin ? float((fB[e + 2] - fB[e + 1]) * inv_h) : 0.f, has_dn ? float((fD[e + 1] - fB[e + 1]) * inv_h) : 0.f,
             e < 0 ? sxbl : f4(sxb, e), e < 0 ? sybl : f4(syb, e), xin, has_dn, nx0, ny0, rx, ry, mx, my);
        RxB[e + 1] = inx ? rx : 0.f;
        RyB[e + 1] = inx ? ry : 0.f;
        if (e >= 0) {
          YxB[e] = nx0;
          YyB[e] = ny0;
          if constexpr (PART) acc[0] += double(pnorm(mx, my, aniso));
          // row a-1: the y component of R only
          cell(f4(yxu, e), f4(yyu, e), xin ? float((fU[e + 1] - fU[e]) * inv_h) : 0.f,
               float((fA[e + 1] - fU[e]) * inv_h), f4(sxu, e), f4(syu, e), xin, true, nx0, ny0, rx, ry, mx, my);
          RyU[e] = has_up ? ry : 0.f;
        }
      }
      st4(y_out + oa + c, make_float4(YxA[0], YxA[1], YxA[2], YxA[3]));
      st4(y_out + n + oa + c, make_float4(YyA[0], YyA[1], YyA[2], YyA[3]));
      st4(y_out + ob + c, make_float4(YxB[0], YxB[1], YxB[2], YxB[3]));
      st4(y_out + n + ob + c, make_float4(YyB[0], YyB[1], YyB[2], YyB[3]));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float dva = (RxA[e + 1] - RxA[e]) + (RyA[e + 1] - RyU[e]);
        const float dvb = (RxB[e + 1] - RxB[e]) + (RyB[e + 1] - RyA[e + 1]);
        mk_put<N, double2>(lds, c + e, -double(dva) * inv_h, -double(dvb) * inv_h);
      }
    }
  } else {
#pragma unroll 1
    for (int m = t; m < N; m += T) lds[lpad(m)] = make_double2(0.0, 0.0);
  }
  if constexpr (PART) group_reduce_store<1, T>(acc, valid ? partials + size_t(a / 2) : nullptr, t);
  __syncthreads();
  Vals<N, double2> v;
  dct2_fwd_lds<N>(t, v, lds, tw, dctw);
  if (valid) {
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      const SlotTile<N> ta(a, t, slot, nyi, lgtw), tb(b, t, slot, nyi, lgtw);
#pragma unroll
      for (int s = 0; s < Sched<N>::H; ++s) {
        rhat[ta.at(s)] = v[slot * Sched<N>::H + s].x;
        rhat[tb.at(s)] = v[slot * Sched<N>::H + s].y;
      }
    }
  }
}

// flux of the single-variable form's latest iterate: m = -tau (R(y) - grad phi) + grad psi,
// y the field the last A read and phi the potential it read; p = proj(y_latest) into pout
// when y_latest is given.  Tall batch layout: y-neighbours stop at instance edges.
__global__ __launch_bounds__(256) void k_emd_finish_drs(const float* __restrict__ y, const double* __restrict__ phi,
                                                        const float* __restrict__ gpsi, float* __restrict__ mout,
                                                        int ny, int nx, int nyi, double inv_h, float tau, int aniso) {
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const bool hx = j < nx - 1, hy = i % nyi < nyi - 1;
    const double fc = phi[o];
    const float gx = hx ? float((phi[o + 1] - fc) * inv_h) : 0.f;
    const float gy = hy ? float((phi[o + nx] - fc) * inv_h) : 0.f;
    const float yx = y[o], yy = y[o + n];
    float qx = yx, qy = yy;
    proj_ball(qx, qy, aniso);
    mout[o] = hx ? -tau * ((2.f * qx - yx) - gx) + gpsi[o] : 0.f;
    mout[o + n] = hy ? -tau * ((2.f * qy - yy) - gy) + gpsi[o + n] : 0.f;
  }
}

// p = proj(y) for a planar 2-component field of n cells
__global__ __launch_bounds__(256) void k_proj2(const float* __restrict__ y, float* __restrict__ p, size_t n,
                                               int aniso) {
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    float qx = y[o], qy = y[o + n];
    proj_ball(qx, qy, aniso);
    p[o] = qx;
    p[o + n] = qy;
  }
}

// ---------------------------------------------------------------- EMD finish
// m = wt - grad phi; if pout: p_out = proj(p_in + sigma m), pbar = 2 p_out - p_in;
// u = m - grad psi (if u); flux = m (if mout).  Pointwise in p (p_in may alias
// p_out or pbar).  Tall batch layout: y-neighbours stop at instance edges.
__global__ __launch_bounds__(256) void k_emd_finish(const float* __restrict__ wt, const double* __restrict__ phi,
                                                    const float* pin, const float* __restrict__ gpsi, float* pout,
                                                    float* pbar, float* __restrict__ u, float* __restrict__ mout,
                                                    int ny, int nx, int nyi, double inv_h, float sigma, int aniso) {
  const size_t n = size_t(ny) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < n; o += size_t(gridDim.x) * blockDim.x) {
    const int i = int(o / nx), j = int(o - size_t(i) * nx);
    const double fc = phi[o];
    const float mx = (j < nx - 1) ? wt[o] - float((phi[o + 1] - fc) * inv_h) : 0.f;
    const float my = (i % nyi < nyi - 1) ? wt[o + n] - float((phi[o + nx] - fc) * inv_h) : 0.f;
    if (pout) {
      const float ox = pin[o], oy = pin[o + n];
      float qx = ox + sigma * mx, qy = oy + sigma * my;
      proj_ball(qx, qy, aniso);
      pout[o] = qx;
      pout[o + n] = qy;
      pbar[o] = 2.f * qx - ox;
      pbar[o + n] = 2.f * qy - oy;
    }
    if (u) {
      u[o] = mx - gpsi[o];
      u[o + n] = my - gpsi[o + n];
    }
    if (mout) {
      mout[o] = mx;
      mout[o + n] = my;
    }
  }
}

}  // namespace gp
