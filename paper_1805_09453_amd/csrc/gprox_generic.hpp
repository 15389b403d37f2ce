// Transforms and iteration kernels for grid sides that are not powers of two.
//
// The Neumann Laplace inversion of the G-prox u-step (appendix A: after even
// reflection the inversion is a cosine series) needs a DCT-II of any length n.
// As in the power-of-two path, a DCT-II of length n is one complex FFT of
// length n over two real sequences packed as (re, im) after Makhoul's
// reordering (v_m = x_{2m} for 2m < n, v_{n-1-m} = x_{2m+1} for 2m + 1 < n;
// X_k = Re(exp(-i pi k / 2n) V_k)); here the FFT is a mixed-radix Stockham
// transform (radices 8, 4, 2, 3, 5, 7, so n must be 7-smooth) running out of
// two LDS buffers, a thread group per row pair, one butterfly per thread and
// pass.  The 2-D solve is row transform -> column transform, diagonal scale
// and inverse column transform (one kernel reading the columns in place) ->
// inverse row transform.  The iteration around it is unfused: separate
// kernels form the right-hand side, update the primal and take the dual step.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/gprox.h"
#include "gprox_fft.hpp"
#include "gprox_kernels.hpp"

namespace gp {

constexpr int kGenMaxPasses = 16;
constexpr int kGenThreads = 256;
// radix schedule of a length: passes in order; per pass the span ns of the
// sub-transforms already done (product of the earlier radices) and M = 2^32 / ns
// rounded up, so that j / ns = umulhi(j, M) for every j < n (exact while j and
// ns are below 2^16; ns = 1 is handled apart)
struct GenSched {
  int n, np;
  int r[kGenMaxPasses];
  int ns[kGenMaxPasses];
  unsigned mg[kGenMaxPasses];
};

// DFT of R points (R = 3, 5, 7) by direct sums, sign exp(-+2 pi i / R)
template <int R, bool INV, class C> __device__ __forceinline__ void dft_small(C* a) {
  using Re = typename Cx<C>::R;
  C y[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    Re xr = a[0].x, xi = a[0].y;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      // angle of W_R^{rs}: compile-time after unrolling
      const int q = (r * s) % R;
      const double ang = (INV ? 2.0 : -2.0) * 3.14159265358979323846 * double(q) / double(R);
      const Re c = Re(__builtin_cos(ang)), sn = Re(__builtin_sin(ang));
      xr += a[r].x * c - a[r].y * sn;
      xi += a[r].x * sn + a[r].y * c;
    }
    y[s] = mk<C>(xr, xi);
  }
#pragma unroll
  for (int s = 0; s < R; ++s) a[s] = y[s];
}

template <int R, bool INV, class C> __device__ __forceinline__ void dft_any(C* a) {
  if constexpr (R == 2 || R == 4 || R == 8) DFT<R, INV, C>::run(a);
  else dft_small<R, INV, C>(a);
}

// One Stockham butterfly of radix R: inputs src[j + r n/R], twiddled by
// W_n^{r k n/(ns R)} (k = j mod ns), outputs dst[(j/ns) ns R + k + r ns].
// W holds W_n^m = exp(-2 pi i m / n), m < n (conjugated for the inverse); the
// twiddle index r k n/(ns R) is below n since r < R and k < ns.
template <int R, bool INV, class C>
__device__ __forceinline__ void gen_bfly(const C* src, C* dst, int j, int n, int ns, unsigned mg, const C* W) {
  const int jq = ns == 1 ? j : int(__umulhi(unsigned(j), mg));
  const int k = j - jq * ns;
  const int step = n / (ns * R);
  C x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    C v = src[j + r * (n / R)];
    if (r > 0 && k > 0) {
      C w = W[r * k * step];
      if (INV) w.y = -w.y;
      v = cmul(v, w);
    }
    x[r] = v;
  }
  dft_any<R, INV, C>(x);
  const int base = jq * ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + r * ns] = x[r];
}

// FFT of the sequence in b0 (length n) by the tid-th of TG threads of a group;
// returns the buffer holding the result.  Every thread of the workgroup calls it
// (it synchronises the workgroup after each pass).
template <bool INV, class C>
__device__ __forceinline__ C* gen_fft(C* b0, C* b1, const GenSched& s, const C* W, int tid, int TG) {
  C* src = b0;
  C* dst = b1;
  for (int p = 0; p < s.np; ++p) {
    const int R = s.r[p], nb = s.n / R, ns = s.ns[p];
    const unsigned mg = s.mg[p];
    for (int j = tid; j < nb; j += TG) {
      switch (R) {
        case 2: gen_bfly<2, INV>(src, dst, j, s.n, ns, mg, W); break;
        case 3: gen_bfly<3, INV>(src, dst, j, s.n, ns, mg, W); break;
        case 4: gen_bfly<4, INV>(src, dst, j, s.n, ns, mg, W); break;
        case 5: gen_bfly<5, INV>(src, dst, j, s.n, ns, mg, W); break;
        case 7: gen_bfly<7, INV>(src, dst, j, s.n, ns, mg, W); break;
        default: gen_bfly<8, INV>(src, dst, j, s.n, ns, mg, W); break;
      }
    }
    __syncthreads();
    C* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Optional right-hand side formed in the loads of a forward row transform
// (mode 0, rows), from a stacked vector field [2][m rows][n] (ntot cells per
// component) in the expressions of the unfused iteration:
//   EMD (FP64): b = -div(u - tau pbar) / h, so that the solve of
//               (0 - Delta) phi = b gives phi = Delta^{-1} div(u - tau pbar);
//   ROF (FP32): r = lt (I - u) + tau_h div pbar  (lt = lambda tau, tau_h = tau / h).
struct GenRhs {
  int kind;  // GP_KIND_ROF or GP_KIND_EMD
  const float* u;
  const float* pb;
  const float* I;
  size_t ntot;
  float tau, lt, tau_h;
  double inv_h;
};
__device__ __forceinline__ double gen_emd_b(const GenRhs& R, size_t o, int i, int j, int rows, int n) {
  const double xr = j < n - 1 ? double(R.u[o]) - double(R.tau) * R.pb[o] : 0.0;
  const double xl = j > 0 ? double(R.u[o - 1]) - double(R.tau) * R.pb[o - 1] : 0.0;
  const double yu = i < rows - 1 ? double(R.u[R.ntot + o]) - double(R.tau) * R.pb[R.ntot + o] : 0.0;
  const double yd = i > 0 ? double(R.u[R.ntot + o - n]) - double(R.tau) * R.pb[R.ntot + o - n] : 0.0;
  return -((xr - xl) + (yu - yd)) * R.inv_h;
}
__device__ __forceinline__ float gen_rof_r(const GenRhs& R, size_t o, int i, int j, int rows, int n) {
  const float xr = j < n - 1 ? R.pb[o] : 0.f, xl = j > 0 ? R.pb[o - 1] : 0.f;
  const float yu = i < rows - 1 ? R.pb[R.ntot + o] : 0.f, yd = i > 0 ? R.pb[R.ntot + o - n] : 0.f;
  return R.lt * (R.I[o] - R.u[o]) + R.tau_h * ((xr - xl) + (yu - yd));
}
template <class Re> __device__ __forceinline__ Re gen_rhs(const GenRhs& R, size_t o, int i, int j, int rows, int n) {
  return R.kind == GP_KIND_EMD ? Re(gen_emd_b(R, o, i, j, rows, n)) : Re(gen_rof_r(R, o, i, j, rows, n));
}

// Row transforms of stacked instances (m instances of `rows` rows of length n,
// row-major, row stride n), or with cols = 1 column transforms (m instances of
// n rows by `rows` columns, row-major: the sequences are the columns, element
// stride `rows`).  A group of TG = blockDim.x / PB threads per row (column) pair
// of an instance (2q, 2q + 1; a lone last one is paired with zeros), PB pairs
// per workgroup, so an instance's results do not depend on the others in the
// stack or on PB.  With WL the twiddle table W is staged in LDS.  A pair is read
// whole before it is written, so in may equal out.  With rh.u set (mode 0, rows)
// the input is the right-hand side formed from the iterates instead of in.
//   mode 0: forward DCT-II, X_k = sum_j x_j cos(pi k (2j + 1) / 2n)
//   mode 1: inverse of it times n (out += result when acc)
//   mode 2: forward, times inv_nn / (alpha + mu_seq[k] + mu_row[row]) (the
//           zero mode dropped where that is 0), inverse times n: the column
//           solve (with cols = 1)
// One workgroup's share (workgroup index bid) of a row or column transform launch.
template <class C, bool WL>
__device__ __forceinline__ void gen_rows_block(const typename Cx<C>::R* in, typename Cx<C>::R* out, int rows, int m,
                                               const GenSched& s, const C* __restrict__ Wg,
                                               const C* __restrict__ dw, const int* __restrict__ active, int mode,
                                               int acc, const typename Cx<C>::R* __restrict__ mu_seq,
                                               const typename Cx<C>::R* __restrict__ mu_row, typename Cx<C>::R alpha,
                                               typename Cx<C>::R inv_nn, int PB, int cols, const GenRhs& rh,
                                               int bid) {
  using Re = typename Cx<C>::R;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = s.n;
  const int TG = blockDim.x / PB, g = threadIdx.x / TG, tid = threadIdx.x - g * TG;
  const int ppi = (rows + 1) / 2;
  // the whole workgroup leaves when none of its row pairs is live
  bool any = false;
  for (int e = 0; e < PB; ++e) {
    const int pe = bid * PB + e, ie = pe / ppi;
    any = any || (ie < m && inst_active(active, ie));
  }
  if (!any) return;
  C* b0 = reinterpret_cast<C*>(smem_raw) + size_t(g) * 2 * n;
  C* b1 = b0 + n;
  const C* W = Wg;
  if constexpr (WL) {
    C* wl = reinterpret_cast<C*>(smem_raw) + size_t(PB) * 2 * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) wl[i] = Wg[i];
    W = wl;  // visible after the barrier below
  }
  const int pair = bid * PB + g;
  const int inst = pair / ppi, q = pair - inst * ppi;
  const bool live = inst < m && inst_active(active, inst);
  const int r0 = 2 * q, r1 = r0 + 1;
  const bool has1 = live && r1 < rows;
  const size_t es = cols ? size_t(rows) : 1;  // element stride of a sequence
  const size_t o0 = !live ? 0 : cols ? size_t(inst) * n * rows + r0 : (size_t(inst) * rows + r0) * n;
  const size_t o1 = !has1 ? o0 : cols ? o0 + 1 : o0 + n;
  if (mode == 1) {
    // Z_k = V^a_k + i V^b_k, V_k = conj(w_k) (X_k - i X_{n-k}), X_n = 0
    for (int k = tid; k < n; k += TG) {
      const Re xa = live ? in[o0 + k * es] : Re(0), xb = has1 ? in[o1 + k * es] : Re(0);
      const Re ya = (k && live) ? in[o0 + (n - k) * es] : Re(0), yb = (k && has1) ? in[o1 + (n - k) * es] : Re(0);
      const C w = mk<C>(dw[k].x, -dw[k].y);
      const C va = cmul(w, mk<C>(xa, -ya)), vb = cmul(w, mk<C>(xb, -yb));
      b0[k] = mk<C>(va.x - vb.y, va.y + vb.x);
    }
  } else {
    for (int j = tid; j < n; j += TG) {
      const int src = j < (n + 1) / 2 ? 2 * j : 2 * (n - 1 - j) + 1;  // Makhoul order
      if (rh.u)  // rows, es = 1
        b0[j] = mk<C>(live ? gen_rhs<Re>(rh, o0 + src, r0, src, rows, n) : Re(0),
                      has1 ? gen_rhs<Re>(rh, o1 + src, r1, src, rows, n) : Re(0));
      else
        b0[j] = mk<C>(live ? in[o0 + src * es] : Re(0), has1 ? in[o1 + src * es] : Re(0));
    }
  }
  __syncthreads();
  C* res;
  if (mode == 1) {
    res = gen_fft<true>(b0, b1, s, W, tid, TG);
  } else {
    res = gen_fft<false>(b0, b1, s, W, tid, TG);
    C* oth = res == b0 ? b1 : b0;
    // split the two real transforms: A_k = (Z_k + conj Z_{n-k}) / 2, B_k = (Z_k - conj Z_{n-k}) / 2i,
    // X_k = Re(w_k A_k); mode 2 scales and re-packs for the inverse
    for (int k = tid; k < n; k += TG) {
      const C z = res[k], zr = res[k ? n - k : 0];
      const C A = mk<C>(Re(0.5) * (z.x + zr.x), Re(0.5) * (z.y - zr.y));
      const C B = mk<C>(Re(0.5) * (z.y + zr.y), Re(-0.5) * (z.x - zr.x));
      Re xa = dw[k].x * A.x - dw[k].y * A.y, xb = dw[k].x * B.x - dw[k].y * B.y;
      if (mode == 0) {
        if (live) out[o0 + k * es] = xa;
        if (has1) out[o1 + k * es] = xb;
      } else {
        const Re da = alpha + mu_seq[k] + mu_row[r0], db = alpha + mu_seq[k] + mu_row[has1 ? r1 : r0];
        xa = da > Re(0) ? xa * (inv_nn / da) : Re(0);
        xb = db > Re(0) ? xb * (inv_nn / db) : Re(0);
        oth[k] = mk<C>(xa, xb);
      }
    }
    if (mode == 0) return;
    __syncthreads();
    for (int k = tid; k < n; k += TG) {
      const C x = oth[k], y = k ? oth[n - k] : mk<C>(Re(0), Re(0));
      const C w = mk<C>(dw[k].x, -dw[k].y);
      const C va = cmul(w, mk<C>(x.x, -y.x)), vb = cmul(w, mk<C>(x.y, -y.y));
      res[k] = mk<C>(va.x - vb.y, va.y + vb.x);
    }
    __syncthreads();
    res = gen_fft<true>(res, oth, s, W, tid, TG);
  }
  // un-Makhoul: x_{2m} = z_m, x_{2m+1} = z_{n-1-m}
  if (!live) return;
  for (int j = tid; j < n; j += TG) {
    const int src = (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
    const C v = res[src];
    if (acc) {
      out[o0 + j * es] += v.x;
      if (has1) out[o1 + j * es] += v.y;
    } else {
      out[o0 + j * es] = v.x;
      if (has1) out[o1 + j * es] = v.y;
    }
  }
}

template <class C, bool WL>
__global__ __launch_bounds__(kGenThreads) void k_gen_rows(const typename Cx<C>::R* in, typename Cx<C>::R* out,
                                                          int rows, int m, GenSched s, const C* __restrict__ Wg,
                                                          const C* __restrict__ dw, const int* __restrict__ active,
                                                          int mode, int acc, const typename Cx<C>::R* __restrict__ mu_seq,
                                                          const typename Cx<C>::R* __restrict__ mu_row,
                                                          typename Cx<C>::R alpha, typename Cx<C>::R inv_nn, int PB,
                                                          int cols, GenRhs rh) {
  gen_rows_block<C, WL>(in, out, rows, m, s, Wg, dw, active, mode, acc, mu_seq, mu_row, alpha, inv_nn, PB, cols, rh,
                        blockIdx.x);
}

// The transforms of several groups (sizes, instance stacks) in one launch: job j
// takes the workgroups [block0_j, block0_{j+1}); its arguments are those of
// k_gen_rows.  Every job runs exactly as it would in a launch of its own.
template <class C> struct GenRowsJob {
  using Re = typename Cx<C>::R;
  GenSched s;
  const Re* in;
  Re* out;
  const C* W;
  const C* dw;
  const int* active;
  const Re* mu_seq;
  const Re* mu_row;
  GenRhs rh;
  Re alpha, inv_nn;
  int rows, m, mode, acc, PB, cols, block0;
};
// the job whose workgroup range holds workgroup b (block0 ascending, jobs[0].block0 = 0)
template <class J> __device__ __forceinline__ int gen_find_job(const J* jobs, int njobs, int b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
template <class C, bool WL>
__global__ __launch_bounds__(kGenThreads) void k_gen_rows_multi(const GenRowsJob<C>* __restrict__ jobs, int njobs) {
  const GenRowsJob<C>& J = jobs[gen_find_job(jobs, njobs, blockIdx.x)];
  gen_rows_block<C, WL>(J.in, J.out, J.rows, J.m, J.s, J.W, J.dw, J.active, J.mode, J.acc, J.mu_seq, J.mu_row, J.alpha,
                        J.inv_nn, J.PB, J.cols, J.rh, blockIdx.x - J.block0);
}

// ---------------------------------------------------------------- iteration kernels
// Cells of m stacked instances of nyi x nx; stencils stop at instance edges.

// ROF dual step p+ = proj(p + sig_h grad u), pbar = 2 p+ - p (pointwise in p)
__device__ __forceinline__ void gen_rof_dual_cells(const float* __restrict__ u, float* __restrict__ p,
                                                   float* __restrict__ pb, int nyi, int nx, int m, float sig_h,
                                                   int aniso, const int* __restrict__ active, int bid, int nblk) {
  const size_t ntot = size_t(m) * nyi * nx, nn = size_t(nyi) * nx;
  for (size_t o = size_t(bid) * blockDim.x + threadIdx.x; o < ntot; o += size_t(nblk) * blockDim.x) {
    const int inst = int(o / nn);
    if (!inst_active(active, inst)) continue;
    const size_t l = o - size_t(inst) * nn;
    const int i = int(l / nx), j = int(l - size_t(i) * nx);
    const float uc = u[o];
    const float gx = j < nx - 1 ? u[o + 1] - uc : 0.f, gy = i < nyi - 1 ? u[o + nx] - uc : 0.f;
    const float ox = p[o], oy = p[ntot + o];
    float qx = ox + sig_h * gx, qy = oy + sig_h * gy;
    proj_ball(qx, qy, aniso);
    p[o] = qx;
    p[ntot + o] = qy;
    pb[o] = 2.f * qx - ox;
    pb[ntot + o] = 2.f * qy - oy;
  }
}

__global__ __launch_bounds__(256) void k_gen_rof_dual(const float* __restrict__ u, float* __restrict__ p,
                                                      float* __restrict__ pb, int nyi, int nx, int m, float sig_h,
                                                      int aniso, const int* __restrict__ active) {
  gen_rof_dual_cells(u, p, pb, nyi, nx, m, sig_h, aniso, active, blockIdx.x, gridDim.x);
}

// The pointwise step of several groups in one launch (as GenRowsJob): the ROF
// dual step (sigma = sig_h) or the EMD update.
struct GenCellJob {
  float *u, *p, *pb;
  const double* phi;
  const float* gpsi;
  const int* active;
  double inv_h;
  float tau, sigma;
  int nyi, nx, m, aniso, block0, nblocks;
};
__global__ __launch_bounds__(256) void k_gen_rof_dual_multi(const GenCellJob* __restrict__ jobs, int njobs) {
  const GenCellJob& J = jobs[gen_find_job(jobs, njobs, blockIdx.x)];
  gen_rof_dual_cells(J.u, J.p, J.pb, J.nyi, J.nx, J.m, J.sigma, J.aniso, J.active, blockIdx.x - J.block0,
                     J.nblocks);
}

// per-instance (blockIdx.y) ROF gap partials [sum |grad u|, sum (u - I)^2, sum I div p, sum (div p)^2]
// (gradients and divergences in 1/h units)
__global__ __launch_bounds__(256) void k_gen_rof_gap(const float* __restrict__ u, const float* __restrict__ p,
                                                     const float* __restrict__ I, int nyi, int nx, int m, int aniso,
                                                     double* __restrict__ partials) {
  const int inst = blockIdx.y;
  const size_t ntot = size_t(m) * nyi * nx, nn = size_t(nyi) * nx, base = size_t(inst) * nn;
  double acc[4] = {0, 0, 0, 0};
  for (size_t l = size_t(blockIdx.x) * blockDim.x + threadIdx.x; l < nn; l += size_t(gridDim.x) * blockDim.x) {
    const size_t o = base + l;
    const int i = int(l / nx), j = int(l - size_t(i) * nx);
    const float uc = u[o];
    const float gx = j < nx - 1 ? u[o + 1] - uc : 0.f, gy = i < nyi - 1 ? u[o + nx] - uc : 0.f;
    const float xr = j < nx - 1 ? p[o] : 0.f, xl = j > 0 ? p[o - 1] : 0.f;
    const float yu = i < nyi - 1 ? p[ntot + o] : 0.f, yd = i > 0 ? p[ntot + o - nx] : 0.f;
    const float d = (xr - xl) + (yu - yd);
    const float e = uc - I[o];
    acc[0] += double(pnorm(gx, gy, aniso));
    acc[1] += double(e) * e;
    acc[2] += double(I[o]) * d;
    acc[3] += double(d) * d;
  }
  const bool mx[4] = {false, false, false, false};
  block_reduce_store<4>(acc, mx, partials + size_t(inst) * gridDim.x * 4);
}

// EMD update, pointwise in u, p, pbar: u+ = (u - tau pbar) - grad phi,
// p+ = proj(p + sigma (u+ + grad psi)), pbar = 2 p+ - p
__device__ __forceinline__ void gen_emd_update_cells(float* __restrict__ u, float* __restrict__ p,
                                                     float* __restrict__ pb, const double* __restrict__ phi,
                                                     const float* __restrict__ gpsi, int nyi, int nx, int m,
                                                     float tau, float sigma, double inv_h, int aniso,
                                                     const int* __restrict__ active, int bid, int nblk) {
  const size_t ntot = size_t(m) * nyi * nx, nn = size_t(nyi) * nx;
  for (size_t o = size_t(bid) * blockDim.x + threadIdx.x; o < ntot; o += size_t(nblk) * blockDim.x) {
    const int inst = int(o / nn);
    if (!inst_active(active, inst)) continue;
    const size_t l = o - size_t(inst) * nn;
    const int i = int(l / nx), j = int(l - size_t(i) * nx);
    const double fc = phi[o];
    const float ux = j < nx - 1 ? float(double(u[o]) - double(tau) * pb[o] - (phi[o + 1] - fc) * inv_h) : 0.f;
    const float uy = i < nyi - 1 ? float(double(u[ntot + o]) - double(tau) * pb[ntot + o] - (phi[o + nx] - fc) * inv_h)
                                 : 0.f;
    u[o] = ux;
    u[ntot + o] = uy;
    const float ox = p[o], oy = p[ntot + o];
    float qx = ox + sigma * (ux + gpsi[o]), qy = oy + sigma * (uy + gpsi[ntot + o]);
    proj_ball(qx, qy, aniso);
    if (j == nx - 1) qx = 0.f;  // no flux through the far faces
    if (i == nyi - 1) qy = 0.f;
    p[o] = qx;
    p[ntot + o] = qy;
    pb[o] = 2.f * qx - ox;
    pb[ntot + o] = 2.f * qy - oy;
  }
}
__global__ __launch_bounds__(256) void k_gen_emd_update(float* __restrict__ u, float* __restrict__ p,
                                                        float* __restrict__ pb, const double* __restrict__ phi,
                                                        const float* __restrict__ gpsi, int nyi, int nx, int m,
                                                        float tau, float sigma, double inv_h, int aniso,
                                                        const int* __restrict__ active) {
  gen_emd_update_cells(u, p, pb, phi, gpsi, nyi, nx, m, tau, sigma, inv_h, aniso, active, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(256) void k_gen_emd_update_multi(const GenCellJob* __restrict__ jobs, int njobs) {
  const GenCellJob& J = jobs[gen_find_job(jobs, njobs, blockIdx.x)];
  gen_emd_update_cells(J.u, J.p, J.pb, J.phi, J.gpsi, J.nyi, J.nx, J.m, J.tau, J.sigma, J.inv_h, J.aniso, J.active,
                       blockIdx.x - J.block0, J.nblocks);
}

// per-instance (blockIdx.y) EMD primal partials [sum |u + grad psi|]; with mout the flux too
__global__ __launch_bounds__(256) void k_gen_emd_primal(const float* __restrict__ u, const float* __restrict__ gpsi,
                                                        float* __restrict__ mout, int nyi, int nx, int m, int aniso,
                                                        double* __restrict__ partials) {
  const int inst = blockIdx.y;
  const size_t ntot = size_t(m) * nyi * nx, nn = size_t(nyi) * nx, base = size_t(inst) * nn;
  double acc[1] = {0};
  for (size_t l = size_t(blockIdx.x) * blockDim.x + threadIdx.x; l < nn; l += size_t(gridDim.x) * blockDim.x) {
    const size_t o = base + l;
    const float mx = u[o] + gpsi[o], my = u[ntot + o] + gpsi[ntot + o];
    if (mout) {
      mout[o] = mx;
      mout[ntot + o] = my;
    }
    acc[0] += double(pnorm(mx, my, aniso));
  }
  const bool mxm[1] = {false};
  block_reduce_store<1>(acc, mxm, partials + size_t(inst) * gridDim.x);
}

// b = -div p / h (FP64) for the certificate potential phi_c = Delta^{-1} div p
__global__ __launch_bounds__(256) void k_gen_div64(const float* __restrict__ p, double* __restrict__ b, int nyi,
                                                   int nx, int m, double inv_h, const int* __restrict__ active) {
  const size_t ntot = size_t(m) * nyi * nx, nn = size_t(nyi) * nx;
  for (size_t o = size_t(blockIdx.x) * blockDim.x + threadIdx.x; o < ntot; o += size_t(gridDim.x) * blockDim.x) {
    const int inst = int(o / nn);
    if (!inst_active(active, inst)) continue;
    const size_t l = o - size_t(inst) * nn;
    const int i = int(l / nx), j = int(l - size_t(i) * nx);
    const double xr = j < nx - 1 ? p[o] : 0.0, xl = j > 0 ? p[o - 1] : 0.0;
    const double yu = i < nyi - 1 ? p[ntot + o] : 0.0, yd = i > 0 ? p[ntot + o - nx] : 0.0;
    b[o] = -((xr - xl) + (yu - yd)) * inv_h;
  }
}

// per-instance (blockIdx.y) certificate partials [sum phi f, max |grad phi|] (1/h units)
__global__ __launch_bounds__(256) void k_gen_emd_cert(const double* __restrict__ phi, const float* __restrict__ f,
                                                      int nyi, int nx, double inv_h, int aniso,
                                                      double* __restrict__ partials) {
  const int inst = blockIdx.y;
  const size_t nn = size_t(nyi) * nx, base = size_t(inst) * nn;
  double acc[2] = {0, 0};
  for (size_t l = size_t(blockIdx.x) * blockDim.x + threadIdx.x; l < nn; l += size_t(gridDim.x) * blockDim.x) {
    const size_t o = base + l;
    const int i = int(l / nx), j = int(l - size_t(i) * nx);
    const double fc = phi[o];
    const double gx = j < nx - 1 ? (phi[o + 1] - fc) * inv_h : 0.0, gy = i < nyi - 1 ? (phi[o + nx] - fc) * inv_h : 0.0;
    acc[0] += fc * double(f[o]);
    acc[1] = fmax(acc[1], aniso ? fmax(fabs(gx), fabs(gy)) : gx * gx + gy * gy);
  }
  if (!aniso) acc[1] = sqrt(acc[1]);
  const bool mx[2] = {false, true};
  block_reduce_store<2>(acc, mx, partials + size_t(inst) * gridDim.x * 2);
}

}  // namespace gp
