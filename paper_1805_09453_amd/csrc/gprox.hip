// libgprox: host orchestration and the C ABI declared in include/gprox.h.
//
// Every solve runs on a Group: m instances of one grid size stacked into tall
// device buffers (btile in gprox_kernels.hpp gives the layout).  The
// single-instance entry points are the m = 1 case; gp_batch_solve groups its
// instances by kind, size, h, lambda and tau, captures chunks of iterations of
// all groups in one hipGraph and retires converged instances between replays
// through per-instance active flags.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/gprox.h"
#include "gprox_fused.hpp"
#include "gprox_generic.hpp"
#include "gprox_kernels.hpp"
#include "ws_unet.hpp"

using namespace gp;

namespace {

constexpr int kMinN = 64, kMaxN = 4096;
// default log2 tile width of the intermediate per precision (FP32, FP64): row
// segments of 64 bytes in both; and the widest tile the tuner tries
constexpr int kTileLgDefault[2] = {4, 3};
constexpr int kTileLgMax = 5;
constexpr int kRedBlocks = 1024;  // partial-sum blocks of the grid-stride reductions
constexpr int kMaxK = 8;
constexpr int kResult = 16;       // doubles in the finalized-result buffers
constexpr int kSideStreams = 8;   // parallel branches of the batch graph

bool is_pow2_in_range(int n) { return n >= kMinN && n <= kMaxN && (n & (n - 1)) == 0; }
int ilog2i(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

struct GenTab {  // per length n of the non-power-of-two path: W_n^m and exp(-i pi m / 2n)
  float2 *w32 = nullptr, *d32 = nullptr;
  double2 *w64 = nullptr, *d64 = nullptr;
};

struct Tables {  // per transform length N
  float2* tw32 = nullptr;
  double2* tw64 = nullptr;
  float2* dw32 = nullptr;  // exp(-i pi k / 2N)
  double2* dw64 = nullptr;
};

}  // namespace

namespace {
struct GenSingle;  // job tables of the single-group iteration on non-power-of-two grids
}
struct gp_ctx {
  hipStream_t stream = nullptr;   // the caller's stream
  hipStream_t bstream = nullptr;  // private stream of gp_batch_solve (graph capture and replay)
  std::vector<hipStream_t> side;  // side streams of the batch graph's parallel branches
  std::vector<hipEvent_t> side_ev;
  hipEvent_t fork_ev = nullptr;
  int max_ny = 0, max_nx = 0;
  Tables tab[13];            // index log2 N
  // launch shapes per [FP32, FP64][log2 N]: FFT groups per block of the row
  // passes (row pairs) and of the column pass (column pairs = half the strip
  // width of the tiled intermediate); defaults, or measured by the autotuner
  int row_g[2][13] = {}, col_g[2][13] = {};
  int col_lw[2][13] = {};  // log2 of the tile width of the intermediate, per column length
  bool row_tuned[2][13] = {}, col_tuned[2][13] = {};
  // the ROF row inverse (kernel B) has its own row-pair count: measured after the
  // joint setting, equal to the row passes' when that is fixed with gp_set_shape
  int rowb_g[13] = {};
  float* work = nullptr;     // [max_n] FP32 tiled intermediate
  float* work2 = nullptr;    // [2 max_n] EMD stored field (ping)
  float* work3 = nullptr;    // [2 max_n] EMD stored field (pong)
  double* work64 = nullptr;  // [2 max_n] FP64 potential and intermediate
  double* partials = nullptr;     // [kRedBlocks * kMaxK]
  double* result = nullptr;       // [kResult] finalized reductions (device)
  double* host_result = nullptr;  // [kResult] pinned
  // eigenvalue tables of -Delta for the single-instance calls (current ny, nx, h)
  float *mux32 = nullptr, *muy32 = nullptr;
  double *mux64 = nullptr, *muy64 = nullptr;
  int mu_ny = -1, mu_nx = -1;
  double mu_h = -1.0;
  // solver arena (grow-only)
  float* arena = nullptr;
  size_t arena_floats = 0;
  // warm-start scratch (grow-only): coarse densities, coarse and fine potential
  float* wsbuf = nullptr;
  size_t wsbuf_floats = 0;
  // non-power-of-two sides: tables per length, solver arena (grow-only)
  std::map<int, GenTab> gtab;
  std::map<int, GenSched> gplan[2];  // radix plan per length [FP32, FP64]: measured or set
  GenSingle* gsingle = nullptr;
  float* garena = nullptr;
  size_t garena_floats = 0;
  // batch arena (grow-only)
  char* barena = nullptr;
  size_t barena_bytes = 0;
  // per-kernel timing (gp_profile)
  bool prof_on = false;
  int prof_arm = -1;  // profiling slot the next GP_LAUNCH times (-1: none)
  std::vector<hipEvent_t> prof_ev;  // 2 per recorded launch
  std::vector<int> prof_id;
  std::vector<double> prof_bytes;
  int prof_used = 0;
  long long prof_dropped[32] = {0};
  char err[512] = {0};
};

namespace {

// kernel kinds for gp_profile
enum KId {
  K_ROWS_FWD, K_COLS, K_ROWS_INV, K_ROWS_FWD64, K_COLS64, K_ROWS_INV64, K_ROF_A, K_ROF_B, K_ROF_FINISH,
  K_EMD_A, K_EMD_B, K_EMD_FINISH, K_DIV64, K_REDUCE, K_GEN_ROWS, K_GEN_ROWS64,
  K_GEN_ROF_DUAL, K_GEN_EMD_UPDATE, K_COUNT
};
const char* kKName[K_COUNT] = {"rows_fwd_dct2", "cols_solve", "rows_inv_dct2", "rows_fwd_dct2_f64",
                               "cols_solve_f64", "rows_inv_dct2_f64", "rof_A_prox_rhs_dct", "rof_B_idct_update",
                               "rof_finish", "emd_A_prox_rhs_dct", "emd_B_idct", "emd_finish", "div_f64",
                               "reduce", "gen_rows_dct", "gen_rows_dct_f64",
                               "gen_rof_dual", "gen_emd_update"};
constexpr int kProfPool = 16384;

// records a start event for a launch of kind id moving `bytes`; returns the slot or -1
// Per-launch timing: prof_begin arms a slot and the next GP_LAUNCH passes the
// slot's two events to hipExtLaunchKernelGGL, which binds them to that kernel's
// own dispatch (start and end timestamps of the kernel, no extra packets in the
// stream: event records between launches would add dispatch gaps to the loop).
int prof_begin(gp_ctx* c, int id, double bytes) {
  if (!c->prof_on) return -1;
  if (c->prof_used >= kProfPool) {
    c->prof_dropped[id]++;
    return -1;
  }
  const int s = c->prof_used++;
  c->prof_id[s] = id;
  c->prof_bytes[s] = bytes;
  c->prof_arm = s;
  return s;
}
void prof_end(gp_ctx* c, int s) {
  if (s >= 0 && c->prof_arm == s) {  // no launch took the slot: drop it
    c->prof_arm = -1;
    c->prof_id[s] = -1;
  }
}

#define GP_LAUNCH(ctx, kernel, grid, block, shmem, stream, ...)                                            \
  do {                                                                                                     \
    if ((ctx)->prof_arm >= 0) {                                                                            \
      const int a_ = (ctx)->prof_arm;                                                                      \
      (ctx)->prof_arm = -1;                                                                                \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, (ctx)->prof_ev[2 * a_],                   \
                            (ctx)->prof_ev[2 * a_ + 1], 0, __VA_ARGS__);                                   \
    } else {                                                                                               \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                                 \
    }                                                                                                      \
  } while (0)

void set_err(gp_ctx* c, const char* fmt, ...) {
  if (!c) return;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(c->err, sizeof(c->err), fmt, ap);
  va_end(ap);
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_err(ctx, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return GP_EHIP;                                                                      \
    }                                                                                      \
  } while (0)

#define LAUNCHCHK(ctx)                                                                     \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) {                                                                \
      set_err(ctx, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
      return GP_EHIP;                                                                      \
    }                                                                                      \
  } while (0)

#define RCHK(expr)       \
  do {                   \
    int rc_ = (expr);    \
    if (rc_) return rc_; \
  } while (0)

int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return int(b < 2048 ? (b ? b : 1) : 2048);
}
int red_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  return int(b < kRedBlocks ? (b ? b : 1) : kRedBlocks);
}

// ---------------------------------------------------------------- tables
template <int N> void fill_tw(std::vector<double>& re, std::vector<double>& im) {
  using S = Sched<N>;
  re.assign(S::total_tw(), 1.0);
  im.assign(S::total_tw(), 0.0);
  // per pass: W_{LS R}^{j} (j < LS) then W_{LS R}^{4 j}; the inverse passes hold the conjugates
  for (int dir = 0; dir < 2; ++dir)
    for (int p = 0; p < S::NP; ++p) {
      const int R = dir ? S::irad(p) : S::rad(p), LS = dir ? S::ils(p) : S::ls(p);
      const int off = dir ? S::itoff(p) : S::toff(p);
      const double sg = dir ? 1.0 : -1.0;
      for (int j = 0; j < LS; ++j) {
        const double a1 = sg * 2.0 * M_PI * double(j) / double(LS * R);
        const double a4 = sg * 2.0 * M_PI * double((4 * j) % (LS * R)) / double(LS * R);
        re[off + j] = cos(a1);
        im[off + j] = sin(a1);
        re[off + LS + j] = cos(a4);
        im[off + LS + j] = sin(a4);
      }
    }
}

void fill_tw_n(int n, std::vector<double>& re, std::vector<double>& im) {
  switch (n) {
    case 64: fill_tw<64>(re, im); break;
    case 128: fill_tw<128>(re, im); break;
    case 256: fill_tw<256>(re, im); break;
    case 512: fill_tw<512>(re, im); break;
    case 1024: fill_tw<1024>(re, im); break;
    case 2048: fill_tw<2048>(re, im); break;
    case 4096: fill_tw<4096>(re, im); break;
  }
}

int build_tables(gp_ctx* c, int n) {
  Tables& T = c->tab[ilog2i(n)];
  if (T.tw32) return GP_OK;
  std::vector<double> re, im;
  fill_tw_n(n, re, im);
  const size_t nt = re.size();
  std::vector<float2> t32(nt);
  std::vector<double2> t64(nt);
  for (size_t i = 0; i < nt; ++i) {
    t32[i] = make_float2(float(re[i]), float(im[i]));
    t64[i] = make_double2(re[i], im[i]);
  }
  std::vector<float2> d32(n);
  std::vector<double2> d64(n);
  for (int k = 0; k < n; ++k) {
    const double a = -M_PI * double(k) / (2.0 * n);
    d32[k] = make_float2(float(cos(a)), float(sin(a)));
    d64[k] = make_double2(cos(a), sin(a));
  }
  HIPCHK(c, hipMalloc(&T.tw32, nt * sizeof(float2)));
  HIPCHK(c, hipMalloc(&T.tw64, nt * sizeof(double2)));
  HIPCHK(c, hipMalloc(&T.dw32, n * sizeof(float2)));
  HIPCHK(c, hipMalloc(&T.dw64, n * sizeof(double2)));
  HIPCHK(c, hipMemcpy(T.tw32, t32.data(), nt * sizeof(float2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(T.tw64, t64.data(), nt * sizeof(double2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(T.dw32, d32.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(T.dw64, d64.data(), n * sizeof(double2), hipMemcpyHostToDevice));
  return GP_OK;
}

// eigenvalues of -Delta along one axis, (4/h^2) sin^2(pi k / 2n), computed in FP64
__global__ void k_mu(double* __restrict__ m64, float* __restrict__ m32, int n, double h) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const double s = sin(M_PI * double(k) / (2.0 * n));
    const double v = 4.0 / (h * h) * s * s;
    m64[k] = v;
    m32[k] = float(v);
  }
}

int fill_mu(gp_ctx* c, double* y64, float* y32, double* x64, float* x32, int ny, int nx, double h) {
  GP_LAUNCH(c, k_mu, dim3((ny + 255) / 256), dim3(256), 0, c->stream, y64, y32, ny, h);
  LAUNCHCHK(c);
  GP_LAUNCH(c, k_mu, dim3((nx + 255) / 256), dim3(256), 0, c->stream, x64, x32, nx, h);
  LAUNCHCHK(c);
  return GP_OK;
}

int set_mu(gp_ctx* c, int ny, int nx, double h) {
  if (c->mu_ny == ny && c->mu_nx == nx && c->mu_h == h) return GP_OK;
  RCHK(fill_mu(c, c->muy64, c->muy32, c->mux64, c->mux32, ny, nx, h));
  c->mu_ny = ny;
  c->mu_nx = nx;
  c->mu_h = h;
  return GP_OK;
}

// ---------------------------------------------------------------- launchers
// shape limits per transform length and precision
struct ShapeInfo {
  int T = 0;                 // threads per FFT group
  int row_def = 0, row_gm = 1, row_gmax = 0;
  int col_def = 0, col_gmax = 0;
  size_t group_lds = 0;      // LDS bytes per group
};
template <class C> ShapeInfo shape_info(int n) {
  ShapeInfo i;
  switch (n) {
#define GP_SI(NN)                                                                                       \
  case NN:                                                                                              \
    i.T = Sched<NN>::T;                                                                                 \
    i.row_def = RowShape<NN, C>::G;                                                                     \
    i.row_gm = RowShape<NN, C>::GM;                                                                     \
    i.row_gmax = RowShape<NN, C>::GMAX;                                                                 \
    i.col_def = ColShape<NN, C>::G;                                                                     \
    i.col_gmax = ColShape<NN, C>::MAXTHREADS / Sched<NN>::T;                                            \
    i.group_lds = RowShape<NN, C>::GROUP_LDS;                                                           \
    break;
    GP_SI(64) GP_SI(128) GP_SI(256) GP_SI(512) GP_SI(1024) GP_SI(2048) GP_SI(4096)
#undef GP_SI
  }
  return i;
}
template <class C> constexpr int prec() { return sizeof(C) == sizeof(double2) ? 1 : 0; }

void init_shapes(gp_ctx* c) {
  for (int ln = 6; ln <= 12; ++ln) {
    const ShapeInfo a = shape_info<float2>(1 << ln), b = shape_info<double2>(1 << ln);
    c->row_g[0][ln] = a.row_def;
    c->rowb_g[ln] = a.row_def;
    c->col_g[0][ln] = a.col_def;
    c->col_lw[0][ln] = kTileLgDefault[0];
    c->col_lw[1][ln] = kTileLgDefault[1];
    c->row_g[1][ln] = b.row_def;
    c->col_g[1][ln] = b.col_def;
  }
}

// column pairs per column-pass block for columns of length ny in a grid nx wide
// (the strip width 2G may not exceed nx)
template <class C> int col_groups(const gp_ctx* c, int ny, int nx) {
  const int G = c->col_g[prec<C>()][ilog2i(ny)];
  return 2 * G > nx ? nx / 2 : G;
}
// log2 of the strip width TW of the tiled intermediate: the stored width, at
// least one column-pass block (2G columns) and at most the grid width.  Row
// kernels store 2 TW-wide segments per row pair and strip, so a wider tile
// gives longer contiguous stores; a column block covers 2G of the TW columns.
template <class C> int col_lgtw(const gp_ctx* c, int ny, int nx) {
  const int lo = ilog2i(2 * col_groups<C>(c, ny, nx)), hi = ilog2i(nx);
  return std::max(lo, std::min(c->col_lw[prec<C>()][ilog2i(ny)], hi));
}

template <class C> const C* tw_of(const Tables& T);
template <> const float2* tw_of<float2>(const Tables& T) { return T.tw32; }
template <> const double2* tw_of<double2>(const Tables& T) { return T.tw64; }
template <class C> const C* dw_of(const Tables& T);
template <> const float2* dw_of<float2>(const Tables& T) { return T.dw32; }
template <> const double2* dw_of<double2>(const Tables& T) { return T.dw64; }

#define GP_DISPATCH_NM(n, T, M, ...)           \
  switch (n) {                                 \
    case 64: T<64>::M(__VA_ARGS__); break;     \
    case 128: T<128>::M(__VA_ARGS__); break;   \
    case 256: T<256>::M(__VA_ARGS__); break;   \
    case 512: T<512>::M(__VA_ARGS__); break;   \
    case 1024: T<1024>::M(__VA_ARGS__); break; \
    case 2048: T<2048>::M(__VA_ARGS__); break; \
    case 4096: T<4096>::M(__VA_ARGS__); break; \
  }

// DCT passes over a stack of m instances of nyi rows
template <class C> struct Pass {
  using Re = typename Cx<C>::R;
  template <int N> struct At {
    static void rows_fwd(gp_ctx* c, const Re* in, Re* out, int nyi, int m, const int* active) {
      const int G = c->row_g[prec<C>()][ilog2i(N)];
      const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
      const Tables& T = c->tab[ilog2i(N)];
      GP_LAUNCH(c, (k_rows_fwd<N, C>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, C>::GROUP_LDS),
                         c->stream, in, out, ny, nyi, active, col_lgtw<C>(c, nyi, N), tw_of<C>(T), dw_of<C>(T));
    }
    static void rows_inv(gp_ctx* c, const Re* in, Re* out, int nyi, int m, const int* active) {
      const int G = c->row_g[prec<C>()][ilog2i(N)];
      const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
      const Tables& T = c->tab[ilog2i(N)];
      GP_LAUNCH(c, (k_rows_inv<N, C>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, C>::GROUP_LDS),
                         c->stream, in, out, ny, nyi, active, col_lgtw<C>(c, nyi, N), tw_of<C>(T), dw_of<C>(T));
    }
    // here N is the column length nyi
    static void cols(gp_ctx* c, Re* buf, int nx, int m, const int* active, const Re* mux, const Re* muy, Re alpha,
                     Re inv_nn) {
      const int G = col_groups<C>(c, N, nx);
      const int blocks = (nx / 2 + G - 1) / G;
      const Tables& T = c->tab[ilog2i(N)];
      GP_LAUNCH(c, (k_cols_solve<N, C>), dim3(blocks, m), dim3(G * Sched<N>::T), (G * ColShape<N, C>::GROUP_LDS),
                         c->stream, buf, nx, active, tw_of<C>(T), dw_of<C>(T), mux, muy, alpha, inv_nn,
                         col_lgtw<C>(c, N, nx));
    }
  };
};
template <int N> using P32 = Pass<float2>::At<N>;
template <int N> using P64 = Pass<double2>::At<N>;

template <int N> struct Fused {
  static void rof_A(gp_ctx* c, const float* u, const float* pin, float* pout, const float* I, float* rhat, int nyi,
                    int m, const int* active, float lt, float tau_h, float sig_h, int aniso, int mode,
                    double* partials) {
    const int G = c->row_g[0][ilog2i(N)];
    const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
    const Tables& T = c->tab[ilog2i(N)];
    // the gap partials are a compile-time variant: without them the accumulators free registers
    if (partials)
      GP_LAUNCH(c, (k_rof_A<N, true>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, float2>::GROUP_LDS),
                c->stream, u, pin, pout, I, rhat, ny, nyi, active, col_lgtw<float2>(c, nyi, N), lt, tau_h, sig_h,
                aniso, mode, partials, T.tw32, T.dw32);
    else
      GP_LAUNCH(c, (k_rof_A<N, false>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, float2>::GROUP_LDS),
                c->stream, u, pin, pout, I, rhat, ny, nyi, active, col_lgtw<float2>(c, nyi, N), lt, tau_h, sig_h,
                aniso, mode, partials, T.tw32, T.dw32);
  }
  static void rof_B(gp_ctx* c, const float* dhat, float* u, int nyi, int m, const int* active) {
    const int G = c->rowb_g[ilog2i(N)];
    const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
    const Tables& T = c->tab[ilog2i(N)];
    GP_LAUNCH(c, (k_rof_B<N>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, float2>::GROUP_LDS),
                       c->stream, dhat, u, ny, nyi, active, col_lgtw<float2>(c, nyi, N), T.tw32, T.dw32);
  }
  static void emd_A(gp_ctx* c, const float* wt_in, const double* phi, const float* pin, const float* gpsi,
                    const float* f, float* pout, float* wt_out, double* rhat, int nyi, int m, const int* active,
                    double inv_h, float tau, float sigma, int aniso, int mode, double* partials) {
    const int G = c->row_g[1][ilog2i(N)];
    const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
    const Tables& T = c->tab[ilog2i(N)];
    if (partials)
      GP_LAUNCH(c, (k_emd_A<N, true>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, double2>::GROUP_LDS),
                c->stream, wt_in, phi, pin, gpsi, f, pout, wt_out, rhat, ny, nyi, active, col_lgtw<double2>(c, nyi, N),
                inv_h, tau, sigma, aniso, mode, partials, T.tw64, T.dw64);
    else
      GP_LAUNCH(c, (k_emd_A<N, false>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, double2>::GROUP_LDS),
                c->stream, wt_in, phi, pin, gpsi, f, pout, wt_out, rhat, ny, nyi, active, col_lgtw<double2>(c, nyi, N),
                inv_h, tau, sigma, aniso, mode, partials, T.tw64, T.dw64);
  }
  static void emd_A_drs(gp_ctx* c, const float* y_in, const double* phi, const float* gpsi, float* y_out,
                        double* rhat, int nyi, int m, const int* active, double inv_h, float tau, float sigma, int aniso,
                        int mode, double* partials) {
    const int G = c->row_g[1][ilog2i(N)];
    const int ny = nyi * m, blocks = (ny / 2 + G - 1) / G;
    const Tables& T = c->tab[ilog2i(N)];
    if (partials)
      GP_LAUNCH(c, (k_emd_A_drs<N, true>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, double2>::GROUP_LDS),
                c->stream, y_in, phi, gpsi, y_out, rhat, ny, nyi, active, col_lgtw<double2>(c, nyi, N), inv_h, tau,
                sigma, aniso, mode, partials, T.tw64, T.dw64);
    else
      GP_LAUNCH(c, (k_emd_A_drs<N, false>), dim3(blocks), dim3(G * Sched<N>::T), (G * RowShape<N, double2>::GROUP_LDS),
                c->stream, y_in, phi, gpsi, y_out, rhat, ny, nyi, active, col_lgtw<double2>(c, nyi, N), inv_h, tau,
                sigma, aniso, mode, partials, T.tw64, T.dw64);
  }
};

// (alpha I - Delta) x = b for m stacked instances: row DCT into the tiled
// intermediate tmp, column solve, row inverse into x.  b and x may alias; tmp must not.
int poisson_f32(gp_ctx* c, const float* b, float* x, int nyi, int nx, int m, const float* mux, const float* muy,
                double alpha, float* tmp) {
  const double fb = 8.0 * double(nx) * nyi * m;  // each pass reads and writes one FP32 field
  int ps = prof_begin(c, K_ROWS_FWD, fb);
  GP_DISPATCH_NM(nx, P32, rows_fwd, c, b, tmp, nyi, m, nullptr);
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_COLS, fb);
  GP_DISPATCH_NM(nyi, P32, cols, c, tmp, nx, m, nullptr, mux, muy, float(alpha), float(1.0 / (double(nx) * nyi)));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROWS_INV, fb);
  GP_DISPATCH_NM(nx, P32, rows_inv, c, tmp, x, nyi, m, nullptr);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}
int poisson_f64(gp_ctx* c, const double* b, double* x, int nyi, int nx, int m, const int* active, const double* mux,
                const double* muy, double alpha, double* tmp) {
  const double fb = 16.0 * double(nx) * nyi * m;
  int ps = prof_begin(c, K_ROWS_FWD64, fb);
  GP_DISPATCH_NM(nx, P64, rows_fwd, c, b, tmp, nyi, m, active);
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_COLS64, fb);
  GP_DISPATCH_NM(nyi, P64, cols, c, tmp, nx, m, active, mux, muy, alpha, 1.0 / (double(nx) * nyi));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROWS_INV64, fb);
  GP_DISPATCH_NM(nx, P64, rows_inv, c, tmp, x, nyi, m, active);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

bool is_side(int n);  // a supported side: 7-smooth in [kMinN, kMaxN] (gprox_generic.inc)

int check_size(gp_ctx* c, int ny, int nx, double h) {
  if (!is_side(ny) || !is_side(nx)) {
    set_err(c, "grid %dx%d unsupported: sides must be in [%d, %d] with no prime factor above 7", ny, nx, kMinN,
            kMaxN);
    return GP_EUNSUPPORTED;
  }
  if (ny > c->max_ny || nx > c->max_nx) {
    set_err(c, "grid %dx%d exceeds the context maximum %dx%d", ny, nx, c->max_ny, c->max_nx);
    return GP_EINVAL;
  }
  if (!(h > 0.0) || !std::isfinite(h)) {
    set_err(c, "h must be positive and finite");
    return GP_EINVAL;
  }
  return GP_OK;
}

int prepare(gp_ctx* c, int ny, int nx, double h) {
  RCHK(check_size(c, ny, nx, h));
  return set_mu(c, ny, nx, h);
}

// finalizes m segments of seg partials (K values each) into c->result and copies
// them to out (synchronises); m * K <= kResult
int finalize_read(gp_ctx* c, const double* partials, int seg, int m, int K, unsigned max_mask, double* out) {
  GP_LAUNCH(c, k_finalize, dim3(m), dim3(256), 0, c->stream, partials, seg, K, max_mask, c->result);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, size_t(m) * K * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < m * K; ++i) out[i] = c->host_result[i];
  return GP_OK;
}

int count_nonfinite(gp_ctx* c, const float* x, size_t n, double* cnt) {
  const int nb = red_blocks(n);
  GP_LAUNCH(c, k_nonfinite, dim3(nb), dim3(256), 0, c->stream, x, n, c->partials);
  LAUNCHCHK(c);
  return finalize_read(c, c->partials, nb, 1, 1, 0u, cnt);
}

float* arena(gp_ctx* c, size_t floats) {
  if (c->arena_floats >= floats) return c->arena;
  if (c->arena) (void)hipFree(c->arena);
  c->arena = nullptr;
  c->arena_floats = 0;
  if (hipMalloc(&c->arena, floats * sizeof(float)) != hipSuccess) {
    c->arena = nullptr;
    return nullptr;
  }
  c->arena_floats = floats;
  return c->arena;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int check_opts(gp_ctx* c, const gp_opts* o, double* tau, double* sigma) {
  if (!o) {
    set_err(c, "opts is NULL");
    return GP_EINVAL;
  }
  *tau = o->tau;
  *sigma = o->sigma > 0 ? o->sigma : 1.0 / o->tau;
  if (!(o->tau > 0) || !std::isfinite(o->tau) || !std::isfinite(*sigma)) {
    set_err(c, "tau must be positive and finite");
    return GP_EINVAL;
  }
  if (*tau * *sigma > 1.0 + 1e-12) {
    set_err(c, "tau * sigma = %g > 1", *tau * *sigma);
    return GP_EINVAL;
  }
  if (o->max_iter < 1 || o->check_every < 1 || !(o->tol >= 0)) {
    set_err(c, "max_iter and check_every must be >= 1 and tol >= 0");
    return GP_EINVAL;
  }
  if (o->norm != GP_NORM_ISO && o->norm != GP_NORM_ANISO) {
    set_err(c, "norm must be GP_NORM_ISO or GP_NORM_ANISO");
    return GP_EINVAL;
  }
  return GP_OK;
}

double rel_gap(double P, double D) { return P != 0.0 ? (P - D) / fabs(P) : fabs(P - D); }

// ---------------------------------------------------------------- groups and pipelines
struct Group {
  int kind = GP_KIND_ROF, nyi = 0, nx = 0, m = 1, norm = GP_NORM_ISO;
  double h = 1, lambda = 0, tau = 1, sigma = 1;
  const float* f = nullptr;     // ROF: the image I; EMD: rho1 - rho0 (mean removed)   [m nyi][nx]
  const float* gpsi = nullptr;  // EMD: grad psi                                       [2][m nyi][nx]
  float *u = nullptr, *p = nullptr, *pbar = nullptr;
  const int* active = nullptr;  // device flag per instance; nullptr: all active
  const float *mux32 = nullptr, *muy32 = nullptr;
  const double *mux64 = nullptr, *muy64 = nullptr;
  float* rhat = nullptr;                     // ROF tiled intermediate [m nyi nx]
  double *rhat64 = nullptr, *phi = nullptr;  // EMD intermediate and potential [m nyi nx]
  float *w0 = nullptr, *w1 = nullptr;        // EMD stored field ping-pong [2][m nyi][nx]
  double* gpart = nullptr;                   // per-row-pair gap partials (ROF 4, EMD 1 per pair)
  size_t ntot() const { return size_t(m) * nyi * nx; }
};

// ROF pipeline.  A(entry) builds rhat from (u_n, pbar_n); each later A advances
// the dual (ping-pong between the two dual buffers) and builds the next rhat.
struct RofPipe {
  gp_ctx* c;
  const Group* g;
  float* X;  // buffer holding the latest complete dual iterate
  float* Y;  // the other dual buffer
};

int rof_A(RofPipe& P, int mode, bool partials) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  const int ps = prof_begin(c, K_ROF_A, (mode == 1 ? 20.0 : 28.0) * double(g.ntot()));
  const float* pin = (mode == 1) ? g.pbar : P.X;
  GP_DISPATCH_NM(g.nx, Fused, rof_A, c, g.u, pin, P.Y, g.f, g.rhat, g.nyi, g.m, g.active, float(g.lambda * g.tau),
                 float(g.tau / g.h), float(g.sigma / g.h), g.norm, mode, partials ? g.gpart : nullptr);
  prof_end(c, ps);
  LAUNCHCHK(c);
  if (mode == 0) std::swap(P.X, P.Y);
  return GP_OK;
}

int rof_CB(RofPipe& P) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  int ps = prof_begin(c, K_COLS, 8.0 * double(g.ntot()));
  GP_DISPATCH_NM(g.nyi, P32, cols, c, g.rhat, g.nx, g.m, g.active, g.mux32, g.muy32, float(g.lambda * g.tau),
                 float(1.0 / (double(g.nyi) * g.nx)));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROF_B, 12.0 * double(g.ntot()));
  GP_DISPATCH_NM(g.nx, Fused, rof_B, c, g.rhat, g.u, g.nyi, g.m, g.active);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

// the state's (p, pbar) from u and the latest dual iterate
int rof_finish(RofPipe& P) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  const int ps = prof_begin(c, K_ROF_FINISH, 28.0 * double(g.ntot()));
  GP_LAUNCH(c, k_rof_finish, dim3(grid_for(g.ntot())), dim3(256), 0, c->stream, g.u, P.X, g.p, g.pbar,
                     g.nyi * g.m, g.nx, g.nyi, float(g.sigma / g.h), g.norm);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

// EMD pipeline: the stored field ping-pongs between w0 and w1, phi and the
// intermediate are FP64.
struct EmdPipe {
  gp_ctx* c;
  const Group* g;
  float *X, *Y;    // dual buffers (X = latest)
  float *WX, *WY;  // stored-field buffers (WX = latest)
};

int emd_A(EmdPipe& P, int mode, bool partials) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  const int ps = prof_begin(c, K_EMD_A, (mode == 1 ? 44.0 : 52.0) * double(g.ntot()));
  const float* win = (mode == 1) ? g.u : P.WX;
  const float* pin = (mode == 1) ? g.pbar : P.X;
  GP_DISPATCH_NM(g.nx, Fused, emd_A, c, win, g.phi, pin, g.gpsi, g.f, P.Y, P.WY, g.rhat64, g.nyi, g.m, g.active,
                 1.0 / g.h, float(g.tau), float(g.sigma), g.norm, mode, partials ? g.gpart : nullptr);
  prof_end(c, ps);
  LAUNCHCHK(c);
  std::swap(P.WX, P.WY);
  if (mode == 0) std::swap(P.X, P.Y);
  return GP_OK;
}

// single-variable form (sigma tau = 1): the y field ping-pongs between WX and WY
// (WX = latest); the entry reads y_0 from the group's u buffer
int emd_A_drs(EmdPipe& P, int mode, bool partials) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  const int ps = prof_begin(c, K_EMD_A, (mode == 1 ? 24.0 : 40.0) * double(g.ntot()));
  const float* yin = (mode == 1) ? g.u : P.WX;
  GP_DISPATCH_NM(g.nx, Fused, emd_A_drs, c, yin, g.phi, g.gpsi, P.WY, g.rhat64, g.nyi, g.m, g.active, 1.0 / g.h,
                 float(g.tau), float(g.sigma), g.norm, mode, partials ? g.gpart : nullptr);
  prof_end(c, ps);
  LAUNCHCHK(c);
  std::swap(P.WX, P.WY);
  return GP_OK;
}

int emd_CB(EmdPipe& P) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  int ps = prof_begin(c, K_COLS64, 16.0 * double(g.ntot()));
  GP_DISPATCH_NM(g.nyi, P64, cols, c, g.rhat64, g.nx, g.m, g.active, g.mux64, g.muy64, 0.0,
                 1.0 / (double(g.nyi) * g.nx));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_EMD_B, 16.0 * double(g.ntot()));
  GP_DISPATCH_NM(g.nx, P64, rows_inv, c, g.rhat64, g.phi, g.nyi, g.m, g.active);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

// m = wt - grad phi; with state: (u, p, pbar) of the state from (wt, phi, latest p);
// with mout: the flux
int emd_finish(EmdPipe& P, const float* wt, bool state, float* mout) {
  gp_ctx* c = P.c;
  const Group& g = *P.g;
  const int ps = prof_begin(c, K_EMD_FINISH, (state ? 56.0 : 24.0) * double(g.ntot()));
  GP_LAUNCH(c, k_emd_finish, dim3(grid_for(g.ntot())), dim3(256), 0, c->stream, wt, g.phi, P.X, g.gpsi,
                     state ? g.p : nullptr, g.pbar, state ? g.u : nullptr, mout, g.nyi * g.m, g.nx, g.nyi, 1.0 / g.h,
                     float(g.sigma), g.norm);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

// EMD certificates of the dual iterates p of all m instances: phi_c = Delta^{-1} div p,
// D = h^2 sum phi_c (rho0 - rho1) / max(1, max |grad phi_c|).  Enqueues only: per
// instance [sum(-phi_c f), max |grad phi_c|] lands in out[2 i], out[2 i + 1].
// phi, tmp: m n doubles (phi is left holding -phi_c; retired instances keep theirs);
// cpart: m * red_blocks(n) * 2.
int emd_cert_enqueue(gp_ctx* c, const Group& g, const float* p, double* phi, double* tmp, double* cpart, double* out) {
  const size_t n = size_t(g.nyi) * g.nx, nt = g.ntot();
  int ps = prof_begin(c, K_DIV64, 16.0 * double(nt));
  const int bx = std::min(256, g.nx);  // the grid widths are powers of two >= 64
  GP_LAUNCH(c, k_div<double>, dim3(g.nx / bx, std::min(g.nyi * g.m, 65535)), dim3(bx), 0, c->stream, p, p + nt,
                     phi, g.nyi * g.m, g.nx, g.nyi, float(1.0 / g.h), g.active);
  prof_end(c, ps);
  LAUNCHCHK(c);
  // Delta phi_c = div p  <=>  (0 I - Delta) phi_c = -div p: solving with div p gives -phi_c
  RCHK(poisson_f64(c, phi, phi, g.nyi, g.nx, g.m, g.active, g.mux64, g.muy64, 0.0, tmp));
  const int nbc = std::min(red_blocks(n), g.nyi);  // row-strided blocks
  ps = prof_begin(c, K_REDUCE, 12.0 * double(nt));
  GP_LAUNCH(c, k_emd_cert, dim3(nbc, g.m), dim3(bx), 0, c->stream, phi, g.f, g.nyi, g.nx, 1.0 / g.h, g.norm,
                     cpart);
  prof_end(c, ps);
  LAUNCHCHK(c);
  GP_LAUNCH(c, k_finalize, dim3(g.m), dim3(256), 0, c->stream, cpart, nbc, 2, 2u, out);
  LAUNCHCHK(c);
  return GP_OK;
}

double emd_dual_from(const double* r, double h) { return h * h * r[0] / (r[1] > 1.0 ? r[1] : 1.0); }

// single-instance Group over a gp_state and the context workspace
Group state_group(gp_ctx* c, const gp_state* s) {
  Group g;
  g.kind = s->kind;
  g.nyi = s->ny;
  g.nx = s->nx;
  g.m = 1;
  g.norm = s->norm;
  g.h = s->h;
  g.lambda = s->lambda;
  g.tau = s->tau;
  g.sigma = s->sigma > 0 ? s->sigma : 1.0 / s->tau;  // sigma <= 0 selects 1/tau, as in gp_opts
  g.f = s->f;
  g.gpsi = s->gpsi;
  g.u = s->u;
  g.p = s->p;
  g.pbar = s->pbar;
  g.mux32 = c->mux32;
  g.muy32 = c->muy32;
  g.mux64 = c->mux64;
  g.muy64 = c->muy64;
  const size_t n = size_t(s->ny) * s->nx;
  g.rhat = c->work;
  g.phi = c->work64;
  g.rhat64 = c->work64 + n;
  g.w0 = c->work3;
  g.w1 = c->work2;
  g.gpart = c->partials;
  return g;
}

// advance (u_n, p_n, pbar_n) by k >= 1 iterations
int rof_advance(gp_ctx* c, const Group& g, int k) {
  RofPipe P{c, &g, g.p, g.pbar};
  RCHK(rof_A(P, 1, false));
  for (int i = 0; i < k; ++i) {
    RCHK(rof_CB(P));
    if (i + 1 < k) RCHK(rof_A(P, 0, false));
  }
  return rof_finish(P);
}

int emd_advance(gp_ctx* c, const Group& g, int k) {
  EmdPipe P{c, &g, g.p, g.pbar, g.w0, g.w1};
  RCHK(emd_A(P, 1, false));
  for (int i = 0; i < k; ++i) {
    RCHK(emd_CB(P));
    if (i + 1 < k) RCHK(emd_A(P, 0, false));
  }
  return emd_finish(P, P.WX, true, nullptr);
}

int rof_gap_state(gp_ctx* c, const gp_state* s, double* P, double* D) {
  const size_t n = size_t(s->ny) * s->nx;
  const int nb = red_blocks(n);
  const int ps = prof_begin(c, K_REDUCE, 16.0 * n);
  GP_LAUNCH(c, k_rof_energy, dim3(nb), dim3(256), 0, c->stream, s->u, s->p, s->p + n, s->f, s->ny, s->nx,
                     float(1.0 / s->h), s->norm, c->partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  double r[4];
  RCHK(finalize_read(c, c->partials, nb, 1, 4, 0u, r));
  const double h2 = s->h * s->h;
  *P = h2 * (r[0] + 0.5 * s->lambda * r[1]);
  *D = -h2 * (r[2] + r[3] / (2.0 * s->lambda));
  return GP_OK;
}

int emd_primal_state(gp_ctx* c, const gp_state* s, double* P) {
  const size_t n = size_t(s->ny) * s->nx;
  const int nb = red_blocks(n);
  GP_LAUNCH(c, k_emd_primal, dim3(nb), dim3(256), 0, c->stream, s->u, s->u + n, s->gpsi, s->gpsi + n, n,
                     s->norm, c->partials);
  LAUNCHCHK(c);
  double r[1];
  RCHK(finalize_read(c, c->partials, nb, 1, 1, 0u, r));
  *P = s->h * s->h * r[0];
  return GP_OK;
}

int validate_state(gp_ctx* c, const gp_state* s) {
  if (!s || !s->f || !s->u || !s->p || !s->pbar || (s->kind == GP_KIND_EMD && !s->gpsi)) {
    set_err(c, "state has a NULL buffer");
    return GP_EINVAL;
  }
  if (s->kind != GP_KIND_ROF && s->kind != GP_KIND_EMD) {
    set_err(c, "state kind must be GP_KIND_ROF or GP_KIND_EMD");
    return GP_EINVAL;
  }
  const double sig = s->sigma > 0 ? s->sigma : 1.0 / s->tau;
  if (!(s->tau > 0) || !std::isfinite(s->tau) || !std::isfinite(sig) || s->tau * sig > 1.0 + 1e-12 ||
      (s->kind == GP_KIND_ROF && !(s->lambda > 0))) {
    set_err(c, "state steps invalid (tau, sigma > 0, tau*sigma <= 1, lambda > 0)");
    return GP_EINVAL;
  }
  if (s->norm != GP_NORM_ISO && s->norm != GP_NORM_ANISO) {
    set_err(c, "state norm invalid");
    return GP_EINVAL;
  }
  return prepare(c, s->ny, s->nx, s->h);
}

// ---------------------------------------------------------------- autotuner
// median time (ms) of `reps` runs of launch() on the context stream, after one warm-up
template <class F> double time_ms(gp_ctx* c, F&& launch, int reps = 3) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return 1e30;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return 1e30;
  }
  launch();
  std::vector<float> ts;
  for (int r = 0; r < reps; ++r) {
    float ms = 1e30f;
    if (hipEventRecord(a, c->stream) == hipSuccess) {
      launch();
      if (hipEventRecord(b, c->stream) == hipSuccess && hipEventSynchronize(b) == hipSuccess)
        (void)hipEventElapsedTime(&ms, a, b);
    }
    ts.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(ts.begin(), ts.end());
  return (hipGetLastError() == hipSuccess) ? ts[ts.size() / 2] : 1e30;
}

#include "gprox_generic.inc"

// Chooses the launch shapes of a group's kernels by measurement.  The column
// setting also fixes the strip width of the tiled intermediate that the row
// passes write and read, so the choice is joint: every (row groups, column
// groups) pair is timed on one iteration's worth of transforms that touch only
// scratch -- the fused row pass in its entry form (reads the state, writes the
// intermediate), the column pass, and the row inverse in place on the
// intermediate.  Results are cached per precision and transform length in the
// context; shapes fixed with gp_set_shape are kept.
int tune_group(gp_ctx* c, const Group& g0) {
  const bool f64 = g0.kind == GP_KIND_EMD;
  const int di = f64 ? 1 : 0, ly = ilog2i(g0.nyi), lx = ilog2i(g0.nx);
  if (c->col_tuned[di][ly] && c->row_tuned[di][lx]) return GP_OK;
  // time a prefix of the stack of at most 16M cells: one steady iteration per
  // candidate (A in its steady mode, the column pass, the row inverse), reading
  // the state and writing only a scratch allocation and the intermediate
  Group g = g0;
  g.m = std::max(1, std::min(g0.m, (1 << 24) / (g0.nyi * g0.nx)));
  const size_t nt = g.ntot();
  float* scr = nullptr;
  if (hipMalloc(&scr, (f64 ? 4 : 2) * nt * sizeof(float)) != hipSuccess) {
    set_err(c, "tuning scratch allocation of %zu bytes failed", (f64 ? 4 : 2) * nt * sizeof(float));
    return GP_ENOMEM;
  }
  const ShapeInfo sy = f64 ? shape_info<double2>(g.nyi) : shape_info<float2>(g.nyi);
  const ShapeInfo sx = f64 ? shape_info<double2>(g.nx) : shape_info<float2>(g.nx);
  std::vector<int> cols, rows, tiles;
  if (c->col_tuned[di][ly]) cols.push_back(c->col_g[di][ly]);
  else
    for (int G = 2; G <= sy.col_gmax && 2 * G <= g.nx; G *= 2) cols.push_back(G);
  if (c->col_tuned[di][ly]) tiles.push_back(c->col_lw[di][ly]);
  else
    for (int l = 2; l <= kTileLgMax && (1 << l) <= g.nx; ++l) tiles.push_back(l);
  if (c->row_tuned[di][lx]) rows.push_back(c->row_g[di][lx]);
  else
    for (int G = sx.row_gm; G <= sx.row_gmax; G *= 2) rows.push_back(G);
  if (cols.empty()) cols.push_back(c->col_g[di][ly]);
  const bool prof = c->prof_on;
  c->prof_on = false;
  double best = 1e30;
  int bc = c->col_g[di][ly], br = c->row_g[di][lx], bl = c->col_lw[di][ly];
  const int dc = bc, dr = br, dl = bl;  // the setting before tuning (the defaults)
  double t_def = 1e30, t_dl = 1e30;       // the defaults; the best at the default tile width
  int dl_c = bc, dl_r = br;
  for (int cg : cols) {
    std::vector<int> lws;  // tile widths below 2G are the same as 2G
    for (int l : tiles) {
      const int e = std::max(l, ilog2i(2 * cg));
      if (lws.empty() || lws.back() != e) lws.push_back(e);
    }
    for (int lw : lws)
      for (int rg : rows) {
        c->col_g[di][ly] = cg;
        c->col_lw[di][ly] = lw;
        c->row_g[di][lx] = rg;
        const double t = time_ms(c, [&] {
          if (f64) {
            // dual and stored field (or y, in the single-variable form the solvers run at
            // sigma tau = 1) to scratch; the potential's row inverse to scratch
            EmdPipe P{c, &g, g.p, scr, g.w0, scr + 2 * nt};
            if (std::fabs(g.sigma * g.tau - 1.0) <= 1e-12)
              (void)emd_A_drs(P, 0, false);
            else
              (void)emd_A(P, 0, false);
            GP_DISPATCH_NM(g.nyi, P64, cols, c, g.rhat64, g.nx, g.m, g.active, g.mux64, g.muy64, 0.0,
                           1.0 / (double(g.nyi) * g.nx));
            GP_DISPATCH_NM(g.nx, P64, rows_inv, c, g.rhat64, reinterpret_cast<double*>(scr), g.nyi, g.m, g.active);
          } else {
            // dual to scratch; the update is applied to a scratch copy of u
            RofPipe P{c, &g, g.p, scr};
            (void)rof_A(P, 0, false);
            GP_DISPATCH_NM(g.nyi, P32, cols, c, g.rhat, g.nx, g.m, g.active, g.mux32, g.muy32, float(g.lambda * g.tau),
                           float(1.0 / (double(g.nyi) * g.nx)));
            GP_DISPATCH_NM(g.nx, Fused, rof_B, c, g.rhat, scr, g.nyi, g.m, g.active);
          }
        }, 7);
        if (lw == std::max(dl, ilog2i(2 * cg))) {
          if (cg == dc && rg == dr) t_def = t;
          if (t < t_dl) {
            t_dl = t;
            dl_c = cg;
            dl_r = rg;
          }
        }
        if (t < best) {
          best = t;
          bc = cg;
          br = rg;
          bl = lw;
        }
      }
  }
  // keep the default tile width, and then the default groups, unless another
  // choice is clearly (3%) faster: single-iteration timings of near-equal
  // shapes differ by a few percent from box to box, and a stable choice keeps
  // runs comparable
  if (t_def <= 1.03 * best) {
    bc = dc;
    br = dr;
    bl = dl;
  } else if (t_dl <= 1.03 * best) {
    bc = dl_c;
    br = dl_r;
    bl = dl;
  }
  c->col_g[di][ly] = bc;
  c->col_lw[di][ly] = bl;
  c->row_g[di][lx] = br;
  if (!f64) c->rowb_g[lx] = br;
  if (!f64 && rows.size() > 1) {
    // the ROF row inverse alone, on the intermediate the last candidate left (its
    // time does not depend on the values), four launches per sample so that the
    // launch overhead does not blur a few percent: kept at the joint choice unless
    // another count is at least 3% faster
    double tb_best = 1e30, tb_joint = 1e30;
    int bb = br;
    for (int rg : rows) {
      c->rowb_g[lx] = rg;
      const double t = time_ms(c, [&] {
        for (int q = 0; q < 4; ++q) GP_DISPATCH_NM(g.nx, Fused, rof_B, c, g.rhat, scr, g.nyi, g.m, g.active);
      }, 7);
      if (rg == br) tb_joint = t;
      if (t < tb_best) {
        tb_best = t;
        bb = rg;
      }
    }
    c->rowb_g[lx] = tb_joint <= 1.03 * tb_best ? br : bb;
  }
  c->col_tuned[di][ly] = true;
  c->row_tuned[di][lx] = true;
  c->prof_on = prof;
  const bool ok = hipGetLastError() == hipSuccess;
  HIPCHK(c, hipFree(scr));
  return ok ? GP_OK : GP_EHIP;
}

// ---------------------------------------------------------------- batch
struct BatchGroup {
  Group g;
  std::vector<int> idx;        // the caller's instance indices, in stack order
  int* active_dev = nullptr;
  float *mu32 = nullptr;       // [nyi + nx]: muy then mux
  double* mu64 = nullptr;
  double* gap_dev = nullptr;   // ROF: [m][4] gap sums; EMD: [m] primal sums
  double* cert_dev = nullptr;  // EMD: [m][2] certificate sums
  double *cphi = nullptr, *ctmp = nullptr, *cpart = nullptr;  // EMD certificate workspace
  float* mflux = nullptr;      // EMD: flux [2][m nyi][nx]
  bool gen = false;            // sides not powers of two: the unfused iteration on gg
  GenGroup gg;
};

// sub-allocator over the batch arena; with base == nullptr it only measures
struct Carver {
  char* base;
  size_t off = 0;
  template <class T> T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

void carve(Carver& A, BatchGroup& bg) {
  Group& g = bg.g;
  const size_t nt = g.ntot(), n = size_t(g.nyi) * g.nx, pairs = size_t(g.m) * g.nyi / 2;
  bg.active_dev = A.take<int>(g.m);
  bg.mu32 = A.take<float>(g.nyi + g.nx);
  bg.mu64 = A.take<double>(g.nyi + g.nx);
  g.active = bg.active_dev;
  g.muy32 = bg.mu32;
  g.mux32 = bg.mu32 ? bg.mu32 + g.nyi : nullptr;
  g.muy64 = bg.mu64;
  g.mux64 = bg.mu64 ? bg.mu64 + g.nyi : nullptr;
  if (bg.gen) {
    GenGroup& q = bg.gg;
    q.kind = g.kind;
    q.nyi = g.nyi;
    q.nx = g.nx;
    q.m = g.m;
    q.norm = g.norm;
    q.h = g.h;
    q.lambda = g.lambda;
    q.tau = g.tau;
    q.sigma = g.sigma;
    q.active = g.active;
    q.muy32 = g.muy32;
    q.mux32 = g.mux32;
    q.muy64 = g.muy64;
    q.mux64 = g.mux64;
    const int nbk = red_blocks(n);
    g.f = q.f = A.take<float>(nt);
    if (g.kind == GP_KIND_ROF) {
      g.u = q.u = A.take<float>(nt);
      g.p = q.p = A.take<float>(2 * nt);
      g.pbar = q.pbar = A.take<float>(2 * nt);
      q.t1 = A.take<float>(nt);
      q.part = A.take<double>(size_t(g.m) * nbk * 4);
      bg.gap_dev = A.take<double>(size_t(g.m) * 4);
    } else {
      g.gpsi = q.gpsi = A.take<float>(2 * nt);
      g.u = q.u = A.take<float>(2 * nt);
      g.p = q.p = A.take<float>(2 * nt);
      g.pbar = q.pbar = A.take<float>(2 * nt);
      q.phi = A.take<double>(nt);
      q.t1d = A.take<double>(nt);
      q.part = A.take<double>(size_t(g.m) * nbk * 2);
      bg.gap_dev = A.take<double>(g.m);
      bg.cert_dev = A.take<double>(size_t(g.m) * 2);
      bg.mflux = A.take<float>(2 * nt);
    }
    return;
  }
  const int vec = g.kind == GP_KIND_ROF ? 1 : 2;  // components of u
  g.f = A.take<float>(nt);
  g.u = A.take<float>(vec * nt);
  g.p = A.take<float>(2 * nt);
  g.pbar = A.take<float>(2 * nt);
  if (g.kind == GP_KIND_ROF) {
    g.rhat = A.take<float>(nt);
    g.gpart = A.take<double>(pairs * 4);
    bg.gap_dev = A.take<double>(size_t(g.m) * 4);
  } else {
    g.gpsi = A.take<float>(2 * nt);
    g.w0 = A.take<float>(2 * nt);
    g.w1 = A.take<float>(2 * nt);
    g.rhat64 = A.take<double>(nt);
    g.phi = A.take<double>(nt);
    bg.cphi = A.take<double>(nt);
    bg.ctmp = A.take<double>(nt);
    g.gpart = A.take<double>(pairs);
    bg.cpart = A.take<double>(size_t(g.m) * red_blocks(n) * 2);
    bg.gap_dev = A.take<double>(g.m);
    bg.cert_dev = A.take<double>(size_t(g.m) * 2);
    bg.mflux = A.take<float>(2 * nt);
  }
}

}  // namespace

// ---------------------------------------------------------------- allocation-free Poisson solve
// dct_poisson_noalloc works without a context and allocates nothing: its
// workspace is the file-scope device array `scratch` below.  In host code the
// array's name is not a device address; the address of each device's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is handed to kernels.
//   layout (bytes):  [0, kNaTiles)              tiled row-transformed field, <= kNaMaxCells floats
//                    then per axis (x, y):      Stockham twiddles (float2), DCT twiddles (float2, N),
//                                               eigenvalues of -Delta (FP64 and FP32, N each)
constexpr size_t kNaMaxCells = size_t(1) << 20;  // ny * nx <= 2^20 (1024 x 1024, 256 x 4096, ...)
constexpr size_t kNaTiles = kNaMaxCells * sizeof(float);
constexpr size_t kNaAxisTw = 4096;               // float2 slots >= Sched<N>::total_tw() for every N
constexpr size_t kNaAxisBytes = kNaAxisTw * sizeof(float2) + size_t(kMaxN) * (sizeof(float2) + sizeof(double) +
                                                                                 sizeof(float));
constexpr size_t kNaBytes = kNaTiles + 2 * kNaAxisBytes;
constexpr int kNaMaxDevices = 64;
static_assert(Sched<4096>::total_tw() <= int(kNaAxisTw) && Sched<512>::total_tw() <= int(kNaAxisTw),
              "twiddle slots");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

std::mutex g_na_mutex;
void* g_na_ptr[kNaMaxDevices] = {};      // device address of `scratch` per device
thread_local char g_na_err[256] = "";   // message of the last failed context-free call

int na_fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_na_err, sizeof(g_na_err), fmt, ap);
  va_end(ap);
  return code;
}

// Stockham twiddles (as build_tables: per direction and pass, W_{LS R}^j for j < LS,
// then W_{LS R}^{4j}; the inverse passes hold the conjugates) and the DCT twiddles
// exp(-i pi k / 2N), from FP64 sincospi on the device, rounded to FP32
template <int N> __global__ __launch_bounds__(256) void k_na_tables(float2* __restrict__ tw, float2* __restrict__ dw) {
  using S = Sched<N>;
  const int stride = int(gridDim.x * blockDim.x);
  for (int k = int(blockIdx.x * blockDim.x + threadIdx.x); k < N; k += stride) {
    double sn, cs;
    sincospi(-double(k) / (2.0 * N), &sn, &cs);
    dw[k] = make_float2(float(cs), float(sn));
  }
  for (int e = int(blockIdx.x * blockDim.x + threadIdx.x); e < S::total_tw(); e += stride) {
    const int dir = e >= S::tsize() ? 1 : 0;
    int p = 0;
    while (p + 1 < S::NP && e >= (dir ? S::itoff(p + 1) : S::toff(p + 1))) ++p;
    const int R = dir ? S::irad(p) : S::rad(p), LS = dir ? S::ils(p) : S::ls(p);
    const int r = e - (dir ? S::itoff(p) : S::toff(p));  // in [0, 2 LS)
    const int j = r < LS ? r : r - LS;
    const int num = r < LS ? j : (4 * j) % (LS * R);
    double sn, cs;
    sincospi((dir ? 2.0 : -2.0) * double(num) / double(LS * R), &sn, &cs);
    tw[e] = make_float2(float(cs), float(sn));
  }
}

struct NaAxis {
  float2* tw;
  float2* dw;
  double* mu64;
  float* mu32;
};
NaAxis na_axis(unsigned char* base, int which) {
  unsigned char* a = base + kNaTiles + size_t(which) * kNaAxisBytes;
  NaAxis x;
  x.tw = reinterpret_cast<float2*>(a);
  x.dw = reinterpret_cast<float2*>(a + kNaAxisTw * sizeof(float2));
  x.mu64 = reinterpret_cast<double*>(a + kNaAxisTw * sizeof(float2) + kMaxN * sizeof(float2));
  x.mu32 = reinterpret_cast<float*>(a + kNaAxisTw * sizeof(float2) + kMaxN * (sizeof(float2) + sizeof(double)));
  return x;
}

// launches of the three passes with the default launch shapes (no tuner state)
template <int N> struct NaPass {
  static void tables(const NaAxis& a, int n, double h, hipStream_t st) {
    hipLaunchKernelGGL((k_na_tables<N>), dim3((N + 255) / 256), dim3(256), 0, st, a.tw, a.dw);
    hipLaunchKernelGGL(k_mu, dim3((n + 255) / 256), dim3(256), 0, st, a.mu64, a.mu32, n, h);
  }
  static void rows_fwd(const NaAxis& a, const float* in, float* out, int ny, int lgtw, hipStream_t st) {
    using SH = RowShape<N, float2>;
    hipLaunchKernelGGL((k_rows_fwd<N, float2>), dim3((ny / 2 + SH::G - 1) / SH::G), dim3(SH::THREADS),
                       SH::LDS_BYTES, st, in, out, ny, ny, nullptr, lgtw, a.tw, a.dw);
  }
  static void rows_inv(const NaAxis& a, const float* in, float* out, int ny, int lgtw, hipStream_t st) {
    using SH = RowShape<N, float2>;
    hipLaunchKernelGGL((k_rows_inv<N, float2>), dim3((ny / 2 + SH::G - 1) / SH::G), dim3(SH::THREADS),
                       SH::LDS_BYTES, st, in, out, ny, ny, nullptr, lgtw, a.tw, a.dw);
  }
  // here N is the column length ny; G column pairs per block (2G <= nx)
  static void cols(const NaAxis& ay, const NaAxis& ax, float* buf, int nx, int G, int lgtw, float alpha,
                   float inv_nn, hipStream_t st) {
    hipLaunchKernelGGL((k_cols_solve<N, float2>), dim3((nx / 2 + G - 1) / G, 1), dim3(G * Sched<N>::T),
                       (size_t(G) * ColShape<N, float2>::GROUP_LDS), st, buf, nx, nullptr, ay.tw, ay.dw, ax.mu32,
                       ay.mu32, alpha, inv_nn, lgtw);
  }
};
template <int N> using NaP = NaPass<N>;
int na_col_groups(int ny) {
  switch (ny) {
#define GP_NA_G(NN) case NN: return ColShape<NN, float2>::G;
    GP_NA_G(64) GP_NA_G(128) GP_NA_G(256) GP_NA_G(512) GP_NA_G(1024) GP_NA_G(2048) GP_NA_G(4096)
#undef GP_NA_G
  }
  return 1;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

const char* gp_strerror(int code) {
  switch (code) {
    case GP_OK: return "ok";
    case GP_ENOTCONV: return "not converged: max_iter reached (outputs valid)";
    case GP_EINVAL: return "invalid argument";
    case GP_EMASS: return "densities have different masses";
    case GP_ENOMEM: return "device allocation failed";
    case GP_EHIP: return "HIP runtime error";
    case GP_EUNSUPPORTED: return "unsupported size or option";
  }
  return "unknown error code";
}

const char* gp_last_error(const gp_ctx* ctx) { return ctx ? ctx->err : g_na_err; }

int gp_create(gp_ctx** out, int max_ny, int max_nx, void* stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  if (!is_side(max_ny) || !is_side(max_nx)) return GP_EUNSUPPORTED;
  gp_ctx* c = new (std::nothrow) gp_ctx();
  if (!c) return GP_ENOMEM;
  c->stream = static_cast<hipStream_t>(stream);
  init_shapes(c);
  c->max_ny = max_ny;
  c->max_nx = max_nx;
  const size_t n = size_t(max_ny) * max_nx;
  bool ok = hipMalloc(&c->work, n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work2, 2 * n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work3, 2 * n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work64, 2 * n * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->partials, size_t(kRedBlocks) * kMaxK * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->result, kResult * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&c->host_result, kResult * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->mux32, kMaxN * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->muy32, kMaxN * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->mux64, kMaxN * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->muy64, kMaxN * sizeof(double)) == hipSuccess;
  if (!ok) {
    gp_destroy(c);
    return GP_ENOMEM;
  }
  for (int nn = kMinN; nn <= kMaxN; nn *= 2) {
    if (nn > max_ny && nn > max_nx) break;
    if (build_tables(c, nn)) {
      gp_destroy(c);
      return GP_EHIP;
    }
  }
  *out = c;
  return GP_OK;
}

int gp_destroy(gp_ctx* c) {
  if (!c) return GP_OK;
  (void)hipStreamSynchronize(c->stream);
  if (c->bstream) {
    (void)hipStreamSynchronize(c->bstream);
    (void)hipStreamDestroy(c->bstream);
  }
  for (auto s : c->side) (void)hipStreamDestroy(s);
  for (auto e : c->side_ev) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  for (auto& T : c->tab) {
    if (T.tw32) (void)hipFree(T.tw32);
    if (T.tw64) (void)hipFree(T.tw64);
    if (T.dw32) (void)hipFree(T.dw32);
    if (T.dw64) (void)hipFree(T.dw64);
  }
  float* fb[] = {c->work, c->work2, c->work3, c->mux32, c->muy32, c->arena};
  for (float* p : fb)
    if (p) (void)hipFree(p);
  double* db[] = {c->work64, c->partials, c->result, c->mux64, c->muy64};
  for (double* p : db)
    if (p) (void)hipFree(p);
  if (c->barena) (void)hipFree(c->barena);
  if (c->wsbuf) (void)hipFree(c->wsbuf);
  if (c->garena) (void)hipFree(c->garena);
  delete c->gsingle;  // frees its job tables
  for (auto& kv : c->gtab) {
    GenTab& T = kv.second;
    void* gb[] = {T.w32, T.d32, T.w64, T.d64};
    for (void* p : gb)
      if (p) (void)hipFree(p);
  }
  for (auto& e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->host_result) (void)hipHostFree(c->host_result);
  delete c;
  return GP_OK;
}

int dct_poisson(gp_ctx* c, const float* b, float* x, int ny, int nx, double h, double alpha) {
  if (!c) return GP_EINVAL;
  if (!b || !x) {
    set_err(c, "NULL buffer");
    return GP_EINVAL;
  }
  if (!(alpha >= 0) || !std::isfinite(alpha)) {
    set_err(c, "alpha must be >= 0 and finite");
    return GP_EINVAL;
  }
  RCHK(prepare(c, ny, nx, h));
  if (is_gen(ny, nx))
    return poisson_gen<float2>(c, b, x, ny, nx, 1, nullptr, c->mux32, c->muy32, alpha, c->work, false);
  return poisson_f32(c, b, x, ny, nx, 1, c->mux32, c->muy32, alpha, c->work);
}

int dct_poisson_noalloc(const float* b, float* x, int ny, int nx, double h, double alpha, void* stream) {
  if (!b || !x) return na_fail(GP_EINVAL, "NULL buffer");
  if (!is_pow2_in_range(ny) || !is_pow2_in_range(nx))
    return na_fail(GP_EUNSUPPORTED, "grid %dx%d unsupported: sides must be powers of two in [%d, %d]", ny, nx,
                   kMinN, kMaxN);
  if (size_t(ny) * size_t(nx) > kNaMaxCells)
    return na_fail(GP_EUNSUPPORTED, "grid %dx%d has %zu cells; dct_poisson_noalloc takes at most %zu", ny, nx,
                   size_t(ny) * size_t(nx), kNaMaxCells);
  if (!(h > 0.0) || !std::isfinite(h)) return na_fail(GP_EINVAL, "h must be positive and finite");
  if (!(alpha >= 0) || !std::isfinite(alpha)) return na_fail(GP_EINVAL, "alpha must be >= 0 and finite");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices)
    return na_fail(GP_EHIP, "no current HIP device (or more than %d devices)", kNaMaxDevices);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_na_mutex);
    if (!g_na_ptr[dev]) {
      // this device's copy of the scratch array; the current device is `dev`
      const hipError_t e = hipGetSymbolAddress(&g_na_ptr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_na_ptr[dev] = nullptr;
        return na_fail(GP_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      }
    }
    base = g_na_ptr[dev];
  }
  unsigned char* sb = static_cast<unsigned char*>(base);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const NaAxis ax = na_axis(sb, 0), ay = na_axis(sb, 1);
  float* tmp = reinterpret_cast<float*>(sb);
  // every table is rewritten by this call (no state survives from an earlier one)
  GP_DISPATCH_NM(nx, NaP, tables, ax, nx, h, st);
  GP_DISPATCH_NM(ny, NaP, tables, ay, ny, h, st);
  const int Gc = std::min(na_col_groups(ny), nx / 2);
  const int lgtw = std::max(ilog2i(2 * Gc), std::min(kTileLgDefault[0], ilog2i(nx)));
  GP_DISPATCH_NM(nx, NaP, rows_fwd, ax, b, tmp, ny, lgtw, st);
  GP_DISPATCH_NM(ny, NaP, cols, ay, ax, tmp, nx, Gc, lgtw, float(alpha), float(1.0 / (double(nx) * ny)), st);
  GP_DISPATCH_NM(nx, NaP, rows_inv, ax, tmp, x, ny, lgtw, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return na_fail(GP_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return GP_OK;
}

int dct_poisson_f64(gp_ctx* c, const double* b, double* x, int ny, int nx, double h, double alpha) {
  if (!c) return GP_EINVAL;
  if (!b || !x) {
    set_err(c, "NULL buffer");
    return GP_EINVAL;
  }
  if (!(alpha >= 0) || !std::isfinite(alpha)) {
    set_err(c, "alpha must be >= 0 and finite");
    return GP_EINVAL;
  }
  RCHK(prepare(c, ny, nx, h));
  if (is_gen(ny, nx))
    return poisson_gen<double2>(c, b, x, ny, nx, 1, nullptr, c->mux64, c->muy64, alpha, c->work64, false);
  return poisson_f64(c, b, x, ny, nx, 1, nullptr, c->mux64, c->muy64, alpha, c->work64);
}

int pd_step(gp_ctx* c, gp_state* s, int n_iter) {
  if (!c) return GP_EINVAL;
  if (n_iter < 0) {
    set_err(c, "n_iter < 0");
    return GP_EINVAL;
  }
  RCHK(validate_state(c, s));
  if (n_iter == 0) return GP_OK;
  if (is_gen(s->ny, s->nx)) {
    const GenGroup g = gen_state_group(c, s);
    for (int i = 0; i < n_iter; ++i) RCHK(gen_single_iter(c, g));
    s->iter += n_iter;
    return GP_OK;
  }
  const Group g = state_group(c, s);
  RCHK(s->kind == GP_KIND_ROF ? rof_advance(c, g, n_iter) : emd_advance(c, g, n_iter));
  s->iter += n_iter;
  return GP_OK;
}

int pd_gap(gp_ctx* c, gp_state* s, gp_report* rep) {
  if (!c) return GP_EINVAL;
  RCHK(validate_state(c, s));
  double P = 0, D = 0;
  if (s->kind == GP_KIND_ROF) {
    RCHK(rof_gap_state(c, s, &P, &D));
  } else {
    RCHK(emd_primal_state(c, s, &P));
    if (is_gen(s->ny, s->nx)) {
      const GenGroup g = gen_state_group(c, s);
      RCHK(gen_emd_values_enqueue(c, g, c->result, c->result + 8, nullptr));
      HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      D = gen_emd_dual(c->host_result + 8, s->h);
    } else {
      // the certificate overwrites the pipeline's phi: the next pd_step starts
      // from the state (its entry step does not read phi)
      const Group g = state_group(c, s);
      const size_t n = size_t(s->ny) * s->nx;
      RCHK(emd_cert_enqueue(c, g, s->p, c->work64, c->work64 + n, c->partials, c->result));
      HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      D = emd_dual_from(c->host_result, s->h);
    }
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->iters = int(s->iter);
    rep->primal = P;
    rep->dual = D;
    rep->rel_gap = rel_gap(P, D);
  }
  return GP_OK;
}

int rof_solve(gp_ctx* c, const float* I, float* u, float* p, int ny, int nx, double h, double lambda,
              const gp_opts* o, gp_report* rep) {
  if (!c) return GP_EINVAL;
  const double t0 = now_s();
  if (!I || !u) {
    set_err(c, "NULL buffer");
    return GP_EINVAL;
  }
  if (!(lambda > 0) || !std::isfinite(lambda)) {
    set_err(c, "lambda must be positive and finite");
    return GP_EINVAL;
  }
  double tau, sigma;
  RCHK(check_opts(c, o, &tau, &sigma));
  RCHK(prepare(c, ny, nx, h));
  const size_t n = size_t(ny) * nx;
  double bad = 0;
  RCHK(count_nonfinite(c, I, n, &bad));
  if (bad > 0) {
    set_err(c, "image has %.0f non-finite values", bad);
    return GP_EINVAL;
  }
  if (is_gen(ny, nx)) {
    if (o->ergodic) {
      set_err(c, "ergodic averages need power-of-two sides");
      return GP_EUNSUPPORTED;
    }
    return rof_solve_gen(c, I, u, p, ny, nx, h, lambda, o, rep, tau, sigma, t0);
  }
  // arena: P0, P1 (2 n floats each); ergodic: sums of u and p (3 n doubles), averages (3 n floats)
  const bool erg = o->ergodic != 0;
  const size_t nar = (erg ? 13 : 4) * n;
  float* ar = arena(c, nar);
  if (!ar) {
    set_err(c, "arena allocation of %zu floats failed", nar);
    return GP_ENOMEM;
  }
  // dual buffers: P0 holds p_0, P1 pbar_0
  float* P0 = ar;
  float* P1 = ar + 2 * n;
  double* esum = reinterpret_cast<double*>(ar + 4 * n);  // [u | px | py] sums
  float* eavg = ar + 10 * n;                             // [u | px | py] averages
  if (o->warm_start && p) {
    HIPCHK(c, hipMemcpyAsync(P0, p, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(c, hipMemsetAsync(P0, 0, 2 * n * sizeof(float), c->stream));
  }
  if (!o->warm_start) HIPCHK(c, hipMemsetAsync(u, 0, n * sizeof(float), c->stream));
  HIPCHK(c, hipMemcpyAsync(P1, P0, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  const gp_state s{GP_KIND_ROF, ny, nx, o->norm, h, lambda, tau, sigma, I, nullptr, u, P0, P1, 0};
  const Group g = state_group(c, &s);
  RCHK(tune_group(c, g));  // launch shapes, measured once per size (reads the state, writes scratch)
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t1 = now_s();
  double P = NAN, D = NAN, gap = NAN;
  bool conv = false;
  int it = 0;
  RofPipe pipe{c, &g, g.p, g.pbar};
  RCHK(rof_A(pipe, 1, false));
  while (it < o->max_iter) {
    RCHK(rof_CB(pipe));  // u_{it+1}
    ++it;
    const bool chk = (it % o->check_every == 0) || (it == o->max_iter);
    // A computes p_it from (u_it, p_{it-1}) and, on checks, the gap partials of (u_it, p_it)
    RCHK(rof_A(pipe, 0, chk && !erg));
    if (erg) {
      // sums of u_1..u_it and p_1..p_it; on checks the gap of their averages
      GP_LAUNCH(c, k_ergodic_add, dim3(grid_for(n / 4)), dim3(256), 0, c->stream,
                reinterpret_cast<const float4*>(g.u), reinterpret_cast<double2*>(esum), n / 4, int(it == 1));
      LAUNCHCHK(c);
      GP_LAUNCH(c, k_ergodic_add, dim3(grid_for(n / 2)), dim3(256), 0, c->stream,
                reinterpret_cast<const float4*>(pipe.X), reinterpret_cast<double2*>(esum + n), n / 2, int(it == 1));
      LAUNCHCHK(c);
    }
    if (chk && erg) {
      GP_LAUNCH(c, k_scale<double>, dim3(grid_for(3 * n)), dim3(256), 0, c->stream, esum, eavg, 3 * n,
                1.0 / double(it));
      LAUNCHCHK(c);
      const gp_state sa{GP_KIND_ROF, ny, nx, o->norm, h, lambda, tau, sigma, I, nullptr, eavg, eavg + n, eavg + n, 0};
      RCHK(rof_gap_state(c, &sa, &P, &D));
    } else if (chk) {
      double r[4];
      RCHK(finalize_read(c, g.gpart, ny / 2, 1, 4, 0u, r));
      P = h * r[0] + 0.5 * lambda * h * h * r[1];
      D = -h * r[2] - r[3] / (2.0 * lambda);
    }
    if (chk) {
      gap = rel_gap(P, D);
      if (!std::isfinite(gap)) {
        set_err(c, "duality gap became non-finite at iteration %d", it);
        return GP_EHIP;
      }
      if (gap <= o->tol) {
        conv = true;
        break;
      }
    }
  }
  if (erg) {
    // the loop ends on a check, so eavg holds the averages over all it iterates
    HIPCHK(c, hipMemcpyAsync(u, eavg, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    if (p) HIPCHK(c, hipMemcpyAsync(p, eavg + n, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  } else if (p) {
    HIPCHK(c, hipMemcpyAsync(p, pipe.X, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t2 = now_s();
  if (rep) {
    rep->iters = it;
    rep->converged = conv;
    rep->primal = P;
    rep->dual = D;
    rep->rel_gap = gap;
    rep->div_residual = 0;
    rep->seconds_setup = t1 - t0;
    rep->seconds_loop = t2 - t1;
  }
  return conv ? GP_OK : GP_ENOTCONV;
}

int emd_setup(gp_ctx* c, const float* rho0, const float* rho1, float* f, float* gpsi, int ny, int nx, double h) {
  if (!c) return GP_EINVAL;
  if (!rho0 || !rho1 || !f || !gpsi) {
    set_err(c, "NULL buffer");
    return GP_EINVAL;
  }
  RCHK(prepare(c, ny, nx, h));
  if (is_gen(ny, nx)) return emd_setup_gen(c, rho0, rho1, f, gpsi, ny, nx, h);
  const size_t n = size_t(ny) * nx;
  const int nb = red_blocks(n);
  GP_LAUNCH(c, k_mass, dim3(nb), dim3(256), 0, c->stream, rho0, rho1, n, c->partials);
  LAUNCHCHK(c);
  double r[3];
  RCHK(finalize_read(c, c->partials, nb, 1, 3, 0u, r));
  const double m0 = r[0], m1 = r[1], bad = r[2];
  if (bad > 0) {
    set_err(c, "densities have %.0f negative or non-finite values", bad);
    return GP_EINVAL;
  }
  if (fabs(m0 - m1) > 1e-6 * fabs(m0)) {
    set_err(c, "mass mismatch: sum rho0 = %.17g, sum rho1 = %.17g", m0, m1);
    return GP_EMASS;
  }
  // c->result still holds [sum rho0, sum rho1] for the FP64 mean
  double* f64 = c->work64;
  double* psi = c->work64;  // the solve consumes f64 before writing psi over it
  double* tmp = c->work64 + n;
  GP_LAUNCH(c, k_f64_diff, dim3(grid_for(n)), dim3(256), 0, c->stream, rho0, rho1, c->result,
                     1.0 / double(n), n, f64, f);
  LAUNCHCHK(c);
  RCHK(poisson_f64(c, f64, psi, ny, nx, 1, nullptr, c->mux64, c->muy64, 0.0, tmp));
  GP_LAUNCH(c, k_grad_f64, dim3(grid_for(n)), dim3(256), 0, c->stream, psi, gpsi, gpsi + n, ny, nx, 1.0 / h);
  LAUNCHCHK(c);
  return GP_OK;
}

int rof_step_rule(gp_ctx* c, const float* I, int ny, int nx, double h, double lambda, double eps, int norm,
                  gp_rof_rule* out) {
  if (!c) return GP_EINVAL;
  if (!I || !out) {
    set_err(c, "NULL argument");
    return GP_EINVAL;
  }
  RCHK(check_size(c, ny, nx, h));
  if (!(lambda > 0) || !std::isfinite(lambda) || !(eps > 0) || !std::isfinite(eps)) {
    set_err(c, "lambda and eps must be positive and finite");
    return GP_EINVAL;
  }
  if (norm != GP_NORM_ISO && norm != GP_NORM_ANISO) {
    set_err(c, "norm must be GP_NORM_ISO or GP_NORM_ANISO");
    return GP_EINVAL;
  }
  const size_t n = size_t(ny) * nx;
  double bad;
  RCHK(count_nonfinite(c, I, n, &bad));
  if (bad > 0) {
    set_err(c, "image has %.0f non-finite values", bad);
    return GP_EINVAL;
  }
  const int nb = red_blocks(n);
  GP_LAUNCH(c, k_rule_sums, dim3(nb), dim3(256), 0, c->stream, I, ny, nx, 1.0 / h, norm, c->partials);
  LAUNCHCHK(c);
  double r[3];
  RCHK(finalize_read(c, c->partials, nb, 1, 3, 0u, r));
  // c->result still holds the three sums: the mean for the centred second moment
  GP_LAUNCH(c, k_centered_sq, dim3(nb), dim3(256), 0, c->stream, I, n, c->result, 1.0 / double(n), c->partials);
  LAUNCHCHK(c);
  double v;
  RCHK(finalize_read(c, c->partials, nb, 1, 1, 0u, &v));
  const double h2 = h * h;
  out->tv = h2 * r[0];
  out->grad_l2 = sqrt(h2 * r[1]);
  out->tv_bound = std::min(out->tv, 0.5 * lambda * h2 * v);
  out->tau_continuum = sqrt(lambda) * out->tv / sqrt(eps);
  out->tau = std::min(out->tau_continuum, out->grad_l2);
  return GP_OK;
}

double emd_step_rule_singular(double eps, double m) {
  if (!(eps > 0) || !(eps < 1) || !(m > 0)) return -1.0;
  return std::min(sqrt(1.0 / (eps * fabs(log(eps)))), 2.0 * pow(m, 0.25));
}

int emd_solve(gp_ctx* c, const float* rho0, const float* rho1, float* m, float* phi, int ny, int nx, double h,
              const gp_opts* o, gp_report* rep) {
  if (!c) return GP_EINVAL;
  const double t0 = now_s();
  if (!rho0 || !rho1 || !m) {
    set_err(c, "NULL buffer");
    return GP_EINVAL;
  }
  double tau, sigma;
  RCHK(check_opts(c, o, &tau, &sigma));
  if (o->warm_start && !phi) {
    set_err(c, "warm_start needs phi");
    return GP_EINVAL;
  }
  RCHK(prepare(c, ny, nx, h));
  if (is_gen(ny, nx)) {
    if (o->ergodic) {
      set_err(c, "ergodic averages need power-of-two sides");
      return GP_EUNSUPPORTED;
    }
    return emd_solve_gen(c, rho0, rho1, m, phi, ny, nx, h, o, rep, tau, sigma, t0);
  }
  const size_t n = size_t(ny) * nx;
  // arena: f, grad psi, u, P0, P1, certificate potential and its intermediate (n doubles each);
  // ergodic: sums of m and p (4 n doubles) and the averaged dual (2 n floats)
  const bool erg = o->ergodic != 0;
  const size_t nar = (erg ? 23 : 13) * n;
  float* ar = arena(c, nar);
  if (!ar) {
    set_err(c, "arena allocation of %zu floats failed", nar);
    return GP_ENOMEM;
  }
  float* f = ar;
  float* gpsi = ar + n;
  float* u = ar + 3 * n;
  float* P0 = ar + 5 * n;
  float* P1 = ar + 7 * n;
  double* cphi = reinterpret_cast<double*>(ar + 9 * n);
  double* ctmp = reinterpret_cast<double*>(ar + 11 * n);
  double* esum = reinterpret_cast<double*>(ar + 13 * n);  // [mx | my | px | py] sums
  float* epavg = ar + 21 * n;                              // [px | py] averages
  RCHK(emd_setup(c, rho0, rho1, f, gpsi, ny, nx, h));
  HIPCHK(c, hipMemsetAsync(u, 0, 2 * n * sizeof(float), c->stream));
  HIPCHK(c, hipMemsetAsync(P0, 0, 2 * n * sizeof(float), c->stream));
  if (o->warm_start) {
    // p0 = proj(grad phi0): the ROF dual step with u = phi0, p = 0, sigma/h = 1/h
    GP_LAUNCH(c, k_rof_finish, dim3(grid_for(n)), dim3(256), 0, c->stream, phi, P0, P0, P1, ny, nx, ny,
                       float(1.0 / h), o->norm);
    LAUNCHCHK(c);
  }
  HIPCHK(c, hipMemcpyAsync(P1, P0, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  const gp_state s{GP_KIND_EMD, ny, nx, o->norm, h, 0.0, tau, sigma, f, gpsi, u, P0, P1, 0};
  const Group g = state_group(c, &s);
  RCHK(tune_group(c, g));  // launch shapes, measured once per size (reads the state, writes scratch)
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t1 = now_s();
  double P = NAN, D = NAN, gap = NAN, L = 0;
  bool conv = false;
  int it = 0;
  // sigma tau = 1 without averaging: the single-variable form (y_0 = p_0 in the u buffer, u_0 = 0
  // being implied); p = proj(y) is formed into P0 on checks
  const bool single = !erg && std::fabs(sigma * tau - 1.0) <= 1e-12;
  if (single) HIPCHK(c, hipMemcpyAsync(u, P0, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  EmdPipe pipe{c, &g, g.p, g.pbar, g.w0, g.w1};
  RCHK(single ? emd_A_drs(pipe, 1, false) : emd_A(pipe, 1, false));
  // device result slots: [0] primal sum, [8..9] certificate sums
  double* cpart = c->partials + size_t(ny / 2);
  while (it < o->max_iter) {
    RCHK(emd_CB(pipe));  // phi_it
    const bool chk = ((it + 1) % o->check_every == 0) || (it + 1 == o->max_iter);
    RCHK(single ? emd_A_drs(pipe, 0, chk) : emd_A(pipe, 0, chk && !erg));  // u_{it+1}, p_{it+1}
    ++it;
    if (erg) {
      // sums of m_1..m_it (m_it = the field A read minus grad phi, now in WY) and p_1..p_it
      GP_LAUNCH(c, k_emd_ergodic_flux, dim3(grid_for(n)), dim3(256), 0, c->stream, pipe.WY, g.phi, esum, ny, nx,
                1.0 / h, int(it == 1));
      LAUNCHCHK(c);
      GP_LAUNCH(c, k_ergodic_add, dim3(grid_for(n / 2)), dim3(256), 0, c->stream,
                reinterpret_cast<const float4*>(pipe.X), reinterpret_cast<double2*>(esum + 2 * n), n / 2,
                int(it == 1));
      LAUNCHCHK(c);
    }
    if (chk) {
      const float* pc = pipe.X;
      if (single) {
        GP_LAUNCH(c, k_proj2, dim3(grid_for(n)), dim3(256), 0, c->stream, pipe.WX, P0, n, o->norm);
        LAUNCHCHK(c);
        pc = P0;
      }
      if (erg) {
        // averaged flux into the caller's m with its primal partials, averaged dual for the certificate
        const int nb = red_blocks(n);
        GP_LAUNCH(c, k_emd_ergodic_primal, dim3(nb), dim3(256), 0, c->stream, esum, 1.0 / double(it), n, o->norm,
                  m, c->partials);
        LAUNCHCHK(c);
        GP_LAUNCH(c, k_finalize, dim3(1), dim3(256), 0, c->stream, c->partials, nb, 1, 0u, c->result);
        LAUNCHCHK(c);
        GP_LAUNCH(c, k_scale<double>, dim3(grid_for(2 * n)), dim3(256), 0, c->stream, esum + 2 * n, epavg, 2 * n,
                  1.0 / double(it));
        LAUNCHCHK(c);
        pc = epavg;
      } else {
        GP_LAUNCH(c, k_finalize, dim3(1), dim3(256), 0, c->stream, g.gpart, ny / 2, 1, 0u, c->result);
        LAUNCHCHK(c);
      }
      // (stream order: the certificate's partials overwrite c->partials only after the finalize above)
      RCHK(emd_cert_enqueue(c, g, pc, cphi, ctmp, cpart, c->result + 8));
      HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      P = h * h * c->host_result[0];
      D = emd_dual_from(c->host_result + 8, h);
      L = c->host_result[9];
      gap = rel_gap(P, D);
      if (!std::isfinite(gap)) {
        set_err(c, "duality gap became non-finite at iteration %d", it);
        return GP_EHIP;
      }
      if (gap <= o->tol) {
        conv = true;
        break;
      }
    }
  }
  // flux m_it = wt_{it-1} - grad phi_{it-1}: the stored field the last A read, now in WY
  // (ergodic: the loop ended on a check, which wrote the averaged flux into m)
  // (single-variable form: m = -tau (R(y) - grad phi) + grad psi from the y the last A read)
  if (single) {
    GP_LAUNCH(c, k_emd_finish_drs, dim3(grid_for(n)), dim3(256), 0, c->stream, pipe.WY, g.phi, gpsi, m, ny, nx, ny,
              1.0 / h, float(tau), o->norm);
    LAUNCHCHK(c);
  } else if (!erg) {
    RCHK(emd_finish(pipe, pipe.WY, false, m));
  }
  if (phi) {
    // cphi holds -phi_c from the last certificate; phi~ = phi_c / max(1, L)
    GP_LAUNCH(c, k_scale<double>, dim3(grid_for(n)), dim3(256), 0, c->stream, cphi, phi, n,
                       -1.0 / (L > 1.0 ? L : 1.0));
    LAUNCHCHK(c);
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t2 = now_s();
  if (rep) {
    rep->iters = it;
    rep->converged = conv;
    rep->primal = P;
    rep->dual = D;
    rep->rel_gap = gap;
    rep->div_residual = 0;
    rep->seconds_setup = t1 - t0;
    rep->seconds_loop = t2 - t1;
  }
  return conv ? GP_OK : GP_ENOTCONV;
}

int gp_batch_solve(gp_ctx* c, const gp_instance* inst, int count, const gp_opts* o, gp_report* reps) {
  if (!c) return GP_EINVAL;
  const double t0 = now_s();
  if (!inst || count < 1 || !o) {
    set_err(c, "batch needs instances (count >= 1) and options");
    return GP_EINVAL;
  }
  if (o->max_iter < 1 || o->check_every < 1 || !(o->tol >= 0) ||
      (o->norm != GP_NORM_ISO && o->norm != GP_NORM_ANISO)) {
    set_err(c, "max_iter and check_every must be >= 1, tol >= 0 and norm valid");
    return GP_EINVAL;
  }
  if (o->ergodic) {
    set_err(c, "ergodic averages are not supported by the batch solver");
    return GP_EUNSUPPORTED;
  }
  if (o->warm_start) {
    set_err(c, "the batch solver starts every instance from zero (warm_start must be 0)");
    return GP_EINVAL;
  }
  // the chunk between checks has an even length, so the ping-pong buffers hold
  // the same roles at every check
  const int C = (o->check_every + 1) / 2 * 2;
  // ---- validate and group
  std::map<std::tuple<int, int, int, double, double, double>, std::vector<int>> groups;
  for (int i = 0; i < count; ++i) {
    const gp_instance& q = inst[i];
    if ((q.kind != GP_KIND_ROF && q.kind != GP_KIND_EMD) || !q.in0 || !q.out ||
        (q.kind == GP_KIND_EMD && !q.in1)) {
      set_err(c, "instance %d: bad kind or NULL buffer", i);
      return GP_EINVAL;
    }
    if (!(q.tau > 0) || !std::isfinite(q.tau) ||
        (q.kind == GP_KIND_ROF && (!(q.lambda > 0) || !std::isfinite(q.lambda)))) {
      set_err(c, "instance %d: tau (and lambda for ROF) must be positive and finite", i);
      return GP_EINVAL;
    }
    const int rc = check_size(c, q.ny, q.nx, q.h);
    if (rc) {
      char msg[512];
      std::snprintf(msg, sizeof(msg), "instance %d: %s", i, c->err);
      std::snprintf(c->err, sizeof(c->err), "%s", msg);
      return rc;
    }
    groups[std::make_tuple(q.kind, q.ny, q.nx, q.h, q.kind == GP_KIND_ROF ? q.lambda : 0.0, q.tau)].push_back(i);
  }
  std::vector<BatchGroup> G;
  for (auto& kv : groups) {
    BatchGroup bg;
    Group& g = bg.g;
    g.kind = std::get<0>(kv.first);
    g.nyi = std::get<1>(kv.first);
    g.nx = std::get<2>(kv.first);
    g.h = std::get<3>(kv.first);
    g.lambda = std::get<4>(kv.first);
    g.tau = std::get<5>(kv.first);
    g.sigma = 1.0 / g.tau;
    g.m = int(kv.second.size());
    g.norm = o->norm;
    bg.idx = kv.second;
    bg.gen = is_gen(g.nyi, g.nx);
    G.push_back(bg);
  }
  // ---- arena
  Carver measure{nullptr};
  for (auto& bg : G) carve(measure, bg);
  if (c->barena_bytes < measure.off) {
    if (c->barena) (void)hipFree(c->barena);
    c->barena = nullptr;
    c->barena_bytes = 0;
    if (hipMalloc(&c->barena, measure.off) != hipSuccess) {
      set_err(c, "batch arena allocation of %zu bytes failed", measure.off);
      return GP_ENOMEM;
    }
    c->barena_bytes = measure.off;
  }
  if (!c->bstream) HIPCHK(c, hipStreamCreateWithFlags(&c->bstream, hipStreamNonBlocking));
  Carver A{c->barena};
  for (auto& bg : G) carve(A, bg);
  // ---- set-up on the caller's stream (outside any graph)
  for (auto& bg : G) {
    Group& g = bg.g;
    const size_t nt = g.ntot(), n = size_t(g.nyi) * g.nx;
    float* f = const_cast<float*>(g.f);
    if (g.kind == GP_KIND_ROF) {
      for (int k = 0; k < g.m; ++k) {
        // a non-finite image is an argument error, as in rof_solve
        double bad;
        RCHK(count_nonfinite(c, inst[bg.idx[k]].in0, n, &bad));
        if (bad > 0) {
          set_err(c, "instance %d: image has %.0f non-finite values", bg.idx[k], bad);
          return GP_EINVAL;
        }
        HIPCHK(c, hipMemcpyAsync(f + k * n, inst[bg.idx[k]].in0, n * sizeof(float), hipMemcpyDeviceToDevice,
                                 c->stream));
      }
      HIPCHK(c, hipMemsetAsync(g.u, 0, nt * sizeof(float), c->stream));
    } else {
      // per instance: FP64 mass check and potential, then scatter grad psi into the stack
      float* gp = const_cast<float*>(g.gpsi);
      for (int k = 0; k < g.m; ++k) {
        const gp_instance& q = inst[bg.idx[k]];
        const int rc = emd_setup(c, q.in0, q.in1, f + k * n, c->work2, g.nyi, g.nx, g.h);
        if (rc) {
          char msg[512];
          std::snprintf(msg, sizeof(msg), "instance %d: %s", bg.idx[k], c->err);
          std::snprintf(c->err, sizeof(c->err), "%s", msg);
          return rc;
        }
        HIPCHK(c, hipMemcpyAsync(gp + k * n, c->work2, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(gp + nt + k * n, c->work2 + n, n * sizeof(float), hipMemcpyDeviceToDevice,
                                 c->stream));
      }
      HIPCHK(c, hipMemsetAsync(g.u, 0, 2 * nt * sizeof(float), c->stream));
    }
    HIPCHK(c, hipMemsetAsync(g.p, 0, 2 * nt * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(g.pbar, 0, 2 * nt * sizeof(float), c->stream));
    std::vector<int> ones(g.m, 1);
    HIPCHK(c, hipMemcpyAsync(bg.active_dev, ones.data(), g.m * sizeof(int), hipMemcpyHostToDevice, c->stream));
    RCHK(fill_mu(c, bg.mu64, bg.mu32, bg.mu64 + g.nyi, bg.mu32 + g.nyi, g.nyi, g.nx, g.h));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // `ones` leaves scope
  }
  // ---- transform tables and radix plans of the non-power-of-two sides (no
  // allocation or measurement inside the capture)
  for (auto& bg : G)
    if (bg.gen) {
      const GenTab* T;
      GenSched sp;
      RCHK(gen_tables(c, bg.g.nyi, &T));
      RCHK(gen_tables(c, bg.g.nx, &T));
      if (bg.g.kind == GP_KIND_EMD) {
        RCHK(gen_plan<double2>(c, bg.g.nyi, &sp));
        RCHK(gen_plan<double2>(c, bg.g.nx, &sp));
      } else {
        RCHK(gen_plan<float2>(c, bg.g.nyi, &sp));
        RCHK(gen_plan<float2>(c, bg.g.nx, &sp));
      }
    }
  // ---- launch shapes: measured per precision and size on first use
  for (auto& bg : G) {
    if (!bg.gen && tune_group(c, bg.g)) {
      set_err(c, "autotuning launch failed");
      return GP_EHIP;
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // ---- pipelines: the entry step eagerly, then one captured chunk of C iterations
  std::vector<RofPipe> rp(G.size());
  std::vector<EmdPipe> ep(G.size());
  for (size_t k = 0; k < G.size(); ++k) {
    const Group& g = G[k].g;
    rp[k] = RofPipe{c, &g, g.p, g.pbar};
    ep[k] = EmdPipe{c, &g, g.p, g.pbar, g.w0, g.w1};
  }
  hipStream_t user = c->stream;
  const bool prof = c->prof_on;
  c->prof_on = false;  // no event records inside a captured graph
  c->stream = c->bstream;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto restore = [&](int r) {
    (void)hipStreamSynchronize(c->bstream);
    c->stream = user;
    c->prof_on = prof;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    return r;
  };
  int rc = GP_OK;
  for (size_t k = 0; k < G.size() && !rc; ++k)
    if (!G[k].gen) rc = G[k].g.kind == GP_KIND_ROF ? rof_A(rp[k], 1, false) : emd_A_drs(ep[k], 1, false);
  if (rc) return restore(rc);
  // side streams: independent groups form parallel branches of the graph
  const int nside = int(std::min<size_t>(G.size(), size_t(kSideStreams))) - 1;
  for (int s = int(c->side.size()); s < nside; ++s) {
    hipStream_t st;
    hipEvent_t ev;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      set_err(c, "side stream creation failed");
      return restore(GP_EHIP);
    }
    c->side.push_back(st);
    c->side_ev.push_back(ev);
  }
  if (!c->fork_ev && hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess) {
    set_err(c, "event creation failed");
    return restore(GP_EHIP);
  }
  // chunk, per group: C x (column pass + B, then A), the last A with gap partials,
  // then the per-instance reductions (ROF: finalize; EMD: finalize + certificate).
  // Only the groups in `live` are captured: the graph is captured again when
  // enough groups have retired completely (their launches would only exit).
  // Every pipeline's buffers return to their roles after the even chunk, so each
  // capture starts from the same state.
  // groups with sides that are not powers of two: per kind, every live group's
  // iteration as one set of launches (job tables written before each capture)
  GenMulti mrof, memd;
  auto build_multi = [&](const std::vector<int>& live) -> int {
    std::vector<const GenGroup*> gr, ge;
    for (int k : live)
      if (G[k].gen) (G[k].g.kind == GP_KIND_ROF ? gr : ge).push_back(&G[k].gg);
    RCHK(gen_multi_build<float2>(c, mrof, GP_KIND_ROF, gr));
    RCHK(gen_multi_build<double2>(c, memd, GP_KIND_EMD, ge));
    return GP_OK;
  };
  auto capture = [&](const std::vector<int>& live) -> int {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    // branches: one per kind for the groups with other sides, one per power-of-two group
    std::vector<int> units;
    if (mrof.nj) units.push_back(-1);
    if (memd.nj) units.push_back(-2);
    for (int k : live)
      if (!G[k].gen) units.push_back(k);
    const int nsd = int(std::min<size_t>(units.size(), size_t(nside + 1))) - 1;
    int rc = GP_OK;
    if (hipStreamBeginCapture(c->bstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      set_err(c, "hipStreamBeginCapture failed");
      return GP_EHIP;
    }
    if (hipEventRecord(c->fork_ev, c->bstream) != hipSuccess) rc = GP_EHIP;
    for (int s = 0; s < nsd && !rc; ++s)
      if (hipStreamWaitEvent(c->side[s], c->fork_ev, 0) != hipSuccess) rc = GP_EHIP;
    if (rc) set_err(c, "fork inside the capture failed");
    for (size_t li = 0; li < units.size() && !rc; ++li) {
      c->stream = li == 0 || nsd == 0 ? c->bstream : c->side[(li - 1) % nsd];
      if (units[li] < 0) {
        // the unfused iteration of every live group of the kind, then per-instance
        // gap values (EMD: primal sums and certificates) group by group
        const int kind = units[li] == -1 ? GP_KIND_ROF : GP_KIND_EMD;
        for (int it = 0; it < C && !rc; ++it)
          rc = kind == GP_KIND_ROF ? gen_multi_iter<float2>(c, mrof) : gen_multi_iter<double2>(c, memd);
        for (int k : live) {
          if (rc || !G[k].gen || G[k].g.kind != kind) continue;
          const GenGroup& q = G[k].gg;
          rc = kind == GP_KIND_ROF ? gen_rof_gap_enqueue(c, q, G[k].gap_dev)
                                   : gen_emd_values_enqueue(c, q, G[k].gap_dev, G[k].cert_dev, nullptr);
        }
        continue;
      }
      const int k = units[li];
      const Group& g = G[k].g;
      for (int it = 0; it < C && !rc; ++it) {
        const bool last = it + 1 == C;
        if (g.kind == GP_KIND_ROF) {
          rc = rof_CB(rp[k]);
          if (!rc) rc = rof_A(rp[k], 0, last);
        } else {
          rc = emd_CB(ep[k]);
          if (!rc) rc = emd_A_drs(ep[k], 0, last);
        }
      }
      if (rc) break;
      GP_LAUNCH(c, k_finalize, dim3(g.m), dim3(256), 0, c->stream, g.gpart, g.nyi / 2,
                g.kind == GP_KIND_ROF ? 4 : 1, 0u, G[k].gap_dev);
      if (hipGetLastError() != hipSuccess) {
        set_err(c, "k_finalize launch failed during capture");
        rc = GP_EHIP;
      }
      if (!rc && g.kind == GP_KIND_EMD) {
        // p = proj(y) of the latest iterate into the (otherwise unused) dual buffer, then its certificate
        GP_LAUNCH(c, k_proj2, dim3(grid_for(g.ntot())), dim3(256), 0, c->stream, ep[k].WX, g.p, g.ntot(), g.norm);
        if (hipGetLastError() != hipSuccess) {
          set_err(c, "k_proj2 launch failed during capture");
          rc = GP_EHIP;
        }
        if (!rc) rc = emd_cert_enqueue(c, g, g.p, G[k].cphi, G[k].ctmp, G[k].cpart, G[k].cert_dev);
      }
    }
    c->stream = c->bstream;
    // join every side stream, also after a failure, so that ending the capture
    // takes all of them out of capture mode
    for (int s = 0; s < nsd; ++s)
      if ((hipEventRecord(c->side_ev[s], c->side[s]) != hipSuccess ||
           hipStreamWaitEvent(c->bstream, c->side_ev[s], 0) != hipSuccess) && !rc) {
        set_err(c, "join inside the capture failed");
        rc = GP_EHIP;
      }
    const hipError_t ce = hipStreamEndCapture(c->bstream, &graph);
    if (rc || ce != hipSuccess) {
      if (!rc) set_err(c, "hipStreamEndCapture failed: %s", hipGetErrorString(ce));
      return rc ? rc : GP_EHIP;
    }
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      set_err(c, "hipGraphInstantiate failed");
      return GP_EHIP;
    }
    return GP_OK;
  };
  std::vector<int> live(G.size());
  for (size_t k = 0; k < G.size(); ++k) live[k] = int(k);
  size_t captured = live.size();
  rc = build_multi(live);
  if (!rc) rc = capture(live);
  if (rc) return restore(rc);
  // ---- replay until every instance has retired
  std::vector<char> retired(count, 0);
  std::vector<int> iters(count, 0);
  std::vector<double> Pv(count, NAN), Dv(count, NAN), gv(count, NAN), tv(count, 0.0), Lv(count, 0.0);
  int left = count, done = 0;
  const double t1 = now_s();
  std::vector<double> hbuf;
  std::vector<int> flags;
  while (left > 0) {
    if (hipGraphLaunch(exec, c->bstream) != hipSuccess) {
      set_err(c, "hipGraphLaunch failed");
      return restore(GP_EHIP);
    }
    done += C;
    for (int k : live) {
      BatchGroup& bg = G[k];
      const Group& g = bg.g;
      const int K = g.kind == GP_KIND_ROF ? 4 : 1;
      hbuf.assign(size_t(g.m) * (K + 2), 0.0);
      if (hipMemcpyAsync(hbuf.data(), bg.gap_dev, size_t(g.m) * K * sizeof(double), hipMemcpyDeviceToHost,
                         c->bstream) != hipSuccess ||
          (g.kind == GP_KIND_EMD &&
           hipMemcpyAsync(hbuf.data() + g.m, bg.cert_dev, size_t(g.m) * 2 * sizeof(double), hipMemcpyDeviceToHost,
                          c->bstream) != hipSuccess) ||
          hipStreamSynchronize(c->bstream) != hipSuccess) {
        set_err(c, "gap read-back failed");
        return restore(GP_EHIP);
      }
      const double now = now_s() - t1;
      flags.assign(g.m, 1);
      bool changed = false;
      for (int k = 0; k < g.m; ++k) {
        const int i = bg.idx[k];
        if (retired[i]) {
          flags[k] = 0;
          continue;
        }
        double P, D;
        if (g.kind == GP_KIND_ROF) {
          const double* r = &hbuf[size_t(k) * 4];
          P = g.h * r[0] + 0.5 * g.lambda * g.h * g.h * r[1];
          D = -g.h * r[2] - r[3] / (2.0 * g.lambda);
        } else {
          P = g.h * g.h * hbuf[k];
          // (the fused path's certificate holds -phi_c, the unfused one phi_c)
          D = bg.gen ? gen_emd_dual(&hbuf[g.m + 2 * size_t(k)], g.h) : emd_dual_from(&hbuf[g.m + 2 * size_t(k)], g.h);
          Lv[i] = hbuf[g.m + 2 * size_t(k) + 1];
        }
        const double gp = rel_gap(P, D);
        Pv[i] = P;
        Dv[i] = D;
        gv[i] = gp;
        iters[i] = done;
        tv[i] = now;
        if (gp <= o->tol || done >= o->max_iter || !std::isfinite(gp)) {
          retired[i] = 1;
          flags[k] = 0;
          --left;
          changed = true;
        }
      }
      if (changed && hipMemcpy(bg.active_dev, flags.data(), g.m * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        set_err(c, "active-flag update failed");
        return restore(GP_EHIP);
      }
    }
    // drop the groups whose instances have all retired; capture again once a
    // quarter of the captured groups are gone
    std::vector<int> still;
    for (int k : live) {
      bool any = false;
      for (int i : G[k].idx) any = any || !retired[i];
      if (any) still.push_back(k);
    }
    live.swap(still);
    if (left > 0 && 4 * live.size() <= 3 * captured) {
      // the replays are done with the job tables before they are rewritten
      if (hipStreamSynchronize(c->bstream) != hipSuccess) {
        set_err(c, "batch stream synchronisation failed");
        return restore(GP_EHIP);
      }
      rc = build_multi(live);
      if (!rc) rc = capture(live);
      if (rc) return restore(rc);
      captured = live.size();
    }
  }
  // ---- outputs: ROF u_t (B never ran after an instance's last check); EMD flux
  // m_t = wt_{t-1} - grad phi_{t-1} (neither was touched after retirement) and,
  // if asked, the scaled certificate potential phi_c / max(1, L) of p_t
  bool ok = true;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    ok = ok && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->bstream) == hipSuccess;
  };
  for (size_t k = 0; k < G.size() && ok; ++k) {
    const BatchGroup& bg = G[k];
    const Group& g = bg.g;
    const size_t n = size_t(g.nyi) * g.nx, nt = g.ntot();
    if (g.kind == GP_KIND_ROF) {
      for (int q = 0; q < g.m; ++q) cp(inst[bg.idx[q]].out, g.u + q * n, n * sizeof(float));
    } else {
      if (bg.gen) {
        // flux m = u + grad psi of the unfused iteration (the primal partials land in scratch)
        GP_LAUNCH(c, k_gen_emd_primal, dim3(bg.gg.nb(), g.m), dim3(256), 0, c->bstream, g.u, g.gpsi, bg.mflux, g.nyi,
                  g.nx, g.m, g.norm, bg.gg.part);
      } else {
        // flux of the single-variable form: m = -tau (R(y) - grad phi) + grad psi from the y the last A read
        GP_LAUNCH(c, k_emd_finish_drs, dim3(grid_for(nt)), dim3(256), 0, c->bstream, ep[k].WY, g.phi, g.gpsi,
                  bg.mflux, g.nyi * g.m, g.nx, g.nyi, 1.0 / g.h, float(g.tau), g.norm);
      }
      if (hipGetLastError() != hipSuccess) {
        set_err(c, "flux kernel launch failed");
        return restore(GP_EHIP);
      }
      for (int q = 0; q < g.m; ++q) {
        const gp_instance& in = inst[bg.idx[q]];
        cp(in.out, bg.mflux + q * n, n * sizeof(float));
        cp(in.out + n, bg.mflux + nt + q * n, n * sizeof(float));
        if (in.phi) {
          const double L = Lv[bg.idx[q]];
          // fused path: cphi holds -phi_c; unfused: phi holds phi_c (each instance's last check)
          const double* src = bg.gen ? bg.gg.phi + q * n : bg.cphi + q * n;
          GP_LAUNCH(c, k_scale<double>, dim3(grid_for(n)), dim3(256), 0, c->bstream, src, in.phi, n,
                    (bg.gen ? 1.0 : -1.0) / (L > 1.0 ? L : 1.0));
          ok = ok && hipGetLastError() == hipSuccess;
        }
      }
    }
  }
  if (!ok || hipStreamSynchronize(c->bstream) != hipSuccess) {
    set_err(c, "batch output copies failed");
    return restore(GP_EHIP);
  }
  bool all_conv = true;
  for (int i = 0; i < count; ++i) {
    const bool conv = gv[i] <= o->tol;
    all_conv = all_conv && conv;
    if (reps) {
      std::memset(&reps[i], 0, sizeof(gp_report));
      reps[i].iters = iters[i];
      reps[i].converged = conv;
      reps[i].primal = Pv[i];
      reps[i].dual = Dv[i];
      reps[i].rel_gap = gv[i];
      reps[i].seconds_setup = t1 - t0;
      reps[i].seconds_loop = tv[i];
    }
  }
  return restore(all_conv ? GP_OK : GP_ENOTCONV);
}

int gp_get_shape(gp_ctx* c, int fp64, int n, int* row_groups, int* col_groups, int* tile_width) {
  if (!c || !is_pow2_in_range(n)) return c ? GP_EUNSUPPORTED : GP_EINVAL;
  const int di = fp64 ? 1 : 0, ln = ilog2i(n);
  if (row_groups) *row_groups = c->row_g[di][ln];
  if (col_groups) *col_groups = c->col_g[di][ln];
  if (tile_width) *tile_width = 1 << c->col_lw[di][ln];
  return GP_OK;
}

int gp_set_shape(gp_ctx* c, int fp64, int n, int row_groups, int col_groups, int tile_width) {
  if (!c) return GP_EINVAL;
  if (!is_pow2_in_range(n)) {
    set_err(c, "n must be a power of two in [%d, %d]", kMinN, kMaxN);
    return GP_EUNSUPPORTED;
  }
  const int di = fp64 ? 1 : 0, ln = ilog2i(n);
  const ShapeInfo si = fp64 ? shape_info<double2>(n) : shape_info<float2>(n);
  if (row_groups && (row_groups < si.row_gm || row_groups > si.row_gmax || row_groups % si.row_gm)) {
    set_err(c, "row groups %d invalid for n=%d (multiples of %d up to %d)", row_groups, n, si.row_gm, si.row_gmax);
    return GP_EINVAL;
  }
  if (col_groups && (col_groups < 1 || col_groups > si.col_gmax || (col_groups & (col_groups - 1)))) {
    set_err(c, "column groups %d invalid for n=%d (powers of two up to %d)", col_groups, n, si.col_gmax);
    return GP_EINVAL;
  }
  if (tile_width && (tile_width < 2 || tile_width > 64 || (tile_width & (tile_width - 1)))) {
    set_err(c, "tile width %d invalid (powers of two in [2, 64])", tile_width);
    return GP_EINVAL;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (row_groups) {
    c->row_g[di][ln] = row_groups;
    c->row_tuned[di][ln] = true;
    if (!fp64) c->rowb_g[ln] = row_groups;
  }
  if (col_groups) c->col_g[di][ln] = col_groups;
  if (tile_width) c->col_lw[di][ln] = ilog2i(tile_width);
  if (col_groups || tile_width) c->col_tuned[di][ln] = true;
  return GP_OK;
}

int gp_get_radix_plan(gp_ctx* c, int fp64, int n, int* radices, int* count) {
  if (!c || !radices || !count) return GP_EINVAL;
  if (!is_side(n) || is_pow2i(n)) {
    set_err(c, "n=%d is not a 7-smooth side in [%d, %d] other than a power of two", n, kMinN, kMaxN);
    return GP_EUNSUPPORTED;
  }
  const auto& P = c->gplan[fp64 ? 1 : 0];
  const auto it = P.find(n);
  const GenSched sp = it != P.end() ? it->second : gen_candidates(n)[0];
  for (int i = 0; i < kGenMaxPasses; ++i) radices[i] = i < sp.np ? sp.r[i] : 0;
  *count = sp.np;
  return GP_OK;
}

int gp_set_radix_plan(gp_ctx* c, int fp64, int n, const int* radices, int count) {
  if (!c || !radices) return GP_EINVAL;
  if (!is_side(n) || is_pow2i(n)) {
    set_err(c, "n=%d is not a 7-smooth side in [%d, %d] other than a power of two", n, kMinN, kMaxN);
    return GP_EUNSUPPORTED;
  }
  if (!valid_plan(n, radices, count)) {
    set_err(c, "radix plan invalid for n=%d (radices 2, 3, 4, 5, 7, 8 with product n, at most %d passes)", n,
            kGenMaxPasses);
    return GP_EINVAL;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  GenSched sp{};
  sp.n = n;
  for (int i = 0; i < count; ++i) sp.r[sp.np++] = radices[i];
  plan_spans(sp);
  c->gplan[fp64 ? 1 : 0][n] = sp;
  // the launch tables of the single-solve path hold the plan they were built with
  gen_single_invalidate(c);
  return GP_OK;
}

// ---------------------------------------------------------------- learned warm start
long long ws_param_count(void) { return wsi::param_count(); }

int ws_create(gp_ctx* c, ws_net** net, int max_batch, int ny, int nx) {
  if (!c || !net) return GP_EINVAL;
  return wsi::create(net, max_batch, ny, nx, c->err, sizeof(c->err));
}

int ws_destroy(ws_net* net) {
  wsi::destroy(net);
  return GP_OK;
}

#define WSCHK(c, net, expr)                                       \
  do {                                                            \
    const int rc_ = (expr);                                       \
    if (rc_) {                                                    \
      std::snprintf((c)->err, sizeof((c)->err), "%s", wsi::error(net)); \
      return rc_;                                                 \
    }                                                             \
  } while (0)

int ws_set_params(gp_ctx* c, ws_net* net, const float* blob) {
  if (!c || !net || !blob) return GP_EINVAL;
  WSCHK(c, net, wsi::set_params(net, c->stream, blob));
  return GP_OK;
}

int ws_get_params(gp_ctx* c, ws_net* net, float* blob) {
  if (!c || !net || !blob) return GP_EINVAL;
  WSCHK(c, net, wsi::get_params(net, c->stream, blob));
  return GP_OK;
}

int ws_predict(gp_ctx* c, ws_net* net, const float* rho0, const float* rho1, int batch, float* phi0) {
  if (!c || !net || !rho0 || !rho1 || !phi0) return GP_EINVAL;
  WSCHK(c, net, wsi::predict(net, c->stream, rho0, rho1, batch, phi0));
  return GP_OK;
}

int ws_grads(gp_ctx* c, ws_net* net, const float* rho0, const float* rho1, const float* phi_star, int batch, double h,
             float* grad, double* loss) {
  if (!c || !net || !rho0 || !rho1 || !phi_star) return GP_EINVAL;
  WSCHK(c, net, wsi::grads(net, c->stream, rho0, rho1, phi_star, batch, h, grad, loss));
  return GP_OK;
}

int ws_adam(gp_ctx* c, ws_net* net, double lr) {
  if (!c || !net || !(lr >= 0) || !std::isfinite(lr)) return GP_EINVAL;
  WSCHK(c, net, wsi::adam(net, c->stream, lr));
  return GP_OK;
}

int ws_train_step(gp_ctx* c, ws_net* net, const float* rho0, const float* rho1, const float* phi_star, int batch,
                  double h, double lr, double* loss) {
  if (!c || !net || !rho0 || !rho1 || !phi_star || !(lr >= 0) || !std::isfinite(lr)) return GP_EINVAL;
  double l = 0.0;
  WSCHK(c, net, wsi::grads(net, c->stream, rho0, rho1, phi_star, batch, h, nullptr, &l));
  WSCHK(c, net, wsi::adam(net, c->stream, lr));
  if (loss) *loss = l;
  return GP_OK;
}

// the parameter blob through a temporary device buffer: load = file -> host ->
// device -> ws_set_params, save = ws_get_params -> device -> host -> file
int ws_load_params(gp_ctx* c, ws_net* net, const char* path) {
  if (!c || !net || !path) return GP_EINVAL;
  const size_t np = size_t(wsi::param_count());
  std::vector<float> h(np);
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    set_err(c, "cannot open %s", path);
    return GP_EINVAL;
  }
  const size_t got = std::fread(h.data(), sizeof(float), np, f);
  const bool more = std::fgetc(f) != EOF;
  std::fclose(f);
  if (got != np || more) {
    set_err(c, "%s does not hold exactly %zu FP32 values", path, np);
    return GP_EINVAL;
  }
  float* d = nullptr;
  if (hipMalloc(&d, np * sizeof(float)) != hipSuccess) {
    set_err(c, "parameter staging allocation of %zu bytes failed", np * sizeof(float));
    return GP_ENOMEM;
  }
  int rc = GP_OK;
  if (hipMemcpyAsync(d, h.data(), np * sizeof(float), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
    set_err(c, "parameter upload failed");
    rc = GP_EHIP;
  } else if (const int r = wsi::set_params(net, c->stream, d)) {
    std::snprintf(c->err, sizeof(c->err), "%s", wsi::error(net));
    rc = r;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && !rc) {
    set_err(c, "parameter upload failed");
    rc = GP_EHIP;
  }
  (void)hipFree(d);
  return rc;
}

int ws_save_params(gp_ctx* c, ws_net* net, const char* path) {
  if (!c || !net || !path) return GP_EINVAL;
  const size_t np = size_t(wsi::param_count());
  std::vector<float> h(np);
  float* d = nullptr;
  if (hipMalloc(&d, np * sizeof(float)) != hipSuccess) {
    set_err(c, "parameter staging allocation of %zu bytes failed", np * sizeof(float));
    return GP_ENOMEM;
  }
  int rc = GP_OK;
  if (const int r = wsi::get_params(net, c->stream, d)) {
    std::snprintf(c->err, sizeof(c->err), "%s", wsi::error(net));
    rc = r;
  } else if (hipMemcpyAsync(h.data(), d, np * sizeof(float), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
             hipStreamSynchronize(c->stream) != hipSuccess) {
    set_err(c, "parameter download failed");
    rc = GP_EHIP;
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (rc) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) {
    set_err(c, "cannot create %s", path);
    return GP_EINVAL;
  }
  const size_t put = std::fwrite(h.data(), sizeof(float), np, f);
  const bool closed = std::fclose(f) == 0;
  if (put != np || !closed) {
    set_err(c, "writing %s failed", path);
    return GP_EINVAL;
  }
  return GP_OK;
}

int ws_downsample(gp_ctx* c, const float* in, int ny, int nx, int f, float* out) {
  if (!c || !in || !out || f < 1 || ny < f || nx < f || ny % f || nx % f) return GP_EINVAL;
  if (wsi::downsample(c->stream, in, ny, nx, f, out)) {
    set_err(c, "downsample launch failed");
    return GP_EHIP;
  }
  return GP_OK;
}

int ws_upsample(gp_ctx* c, const float* in, int ny, int nx, int f, float* out) {
  if (!c || !in || !out || f < 1 || ny < 1 || nx < 1) return GP_EINVAL;
  if (wsi::upsample(c->stream, in, ny, nx, f, out)) {
    set_err(c, "upsample launch failed");
    return GP_EHIP;
  }
  return GP_OK;
}

int ws_emd_solve(gp_ctx* c, ws_net* net, const float* rho0, const float* rho1, float* m, float* phi, int ny, int nx,
                 double h, const gp_opts* o, gp_report* rep, ws_report* wrep) {
  if (!c || !net) return GP_EINVAL;
  const double t0 = now_s();
  if (!rho0 || !rho1 || !m || !o) {
    set_err(c, "NULL argument");
    return GP_EINVAL;
  }
  RCHK(check_size(c, ny, nx, h));
  int H, W, B;
  wsi::native(net, &H, &W, &B);
  const int f = ny / H;
  if (ny % H || nx % W || nx / W != f || (f & (f - 1))) {
    set_err(c, "grid %dx%d is not a power-of-two multiple of the network's %dx%d", ny, nx, H, W);
    return GP_EUNSUPPORTED;
  }
  const size_t n = size_t(ny) * nx, nc = size_t(H) * W;
  const size_t need = 3 * nc + n;
  if (c->wsbuf_floats < need) {
    if (c->wsbuf) (void)hipFree(c->wsbuf);
    c->wsbuf = nullptr;
    c->wsbuf_floats = 0;
    if (hipMalloc(&c->wsbuf, need * sizeof(float)) != hipSuccess) {
      set_err(c, "warm-start scratch allocation failed");
      return GP_ENOMEM;
    }
    c->wsbuf_floats = need;
  }
  float* phi0 = phi ? phi : c->wsbuf + 3 * nc;
  const float *c0 = rho0, *c1 = rho1;
  float* cphi = f > 1 ? c->wsbuf + 2 * nc : phi0;
  if (f > 1) {
    if (wsi::downsample(c->stream, rho0, ny, nx, f, c->wsbuf) || wsi::downsample(c->stream, rho1, ny, nx, f,
                                                                                 c->wsbuf + nc)) {
      set_err(c, "downsample launch failed");
      return GP_EHIP;
    }
    c0 = c->wsbuf;
    c1 = c->wsbuf + nc;
  }
  WSCHK(c, net, wsi::predict(net, c->stream, c0, c1, 1, cphi));
  if (f > 1 && wsi::upsample(c->stream, cphi, H, W, f, phi0)) {
    set_err(c, "upsample launch failed");
    return GP_EHIP;
  }
  // D(phi0): the certificate of the prediction itself
  const int nb = std::min(red_blocks(n), ny);  // row-strided blocks of min(256, nx) threads
  GP_LAUNCH(c, k_phi_cert, dim3(nb), dim3(std::min(256, nx)), 0, c->stream, phi0, rho0, rho1, ny, nx, 1.0 / h,
                     o->norm, c->partials);
  LAUNCHCHK(c);
  double r[2];
  RCHK(finalize_read(c, c->partials, nb, 1, 2, 2u, r));
  ws_report w{};
  w.d0 = h * h * r[0] / (r[1] > 1.0 ? r[1] : 1.0);
  w.seconds_predict = now_s() - t0;
  gp_report r1{};
  int rc = GP_ENOTCONV;
  if (w.d0 > 0.0 && std::isfinite(w.d0)) {
    gp_opts ow = *o;
    ow.warm_start = 1;
    rc = emd_solve(c, rho0, rho1, m, phi0, ny, nx, h, &ow, &r1);
    if (rc != GP_OK && rc != GP_ENOTCONV) return rc;
    w.warm_iters = r1.iters;
    w.used_warm = rc == GP_OK;
  }
  if (!w.used_warm) {
    gp_opts op = *o;
    op.warm_start = 0;
    w.fallback = 1;
    rc = emd_solve(c, rho0, rho1, m, phi, ny, nx, h, &op, &r1);
    if (rc != GP_OK && rc != GP_ENOTCONV) return rc;
  }
  w.seconds_total = now_s() - t0;
  if (rep) *rep = r1;
  if (wrep) *wrep = w;
  return rc;
}

int gp_profile(gp_ctx* c, int enable) {
  if (!c) return GP_EINVAL;
  if (enable) {
    if (c->prof_ev.empty()) {
      c->prof_ev.resize(2 * kProfPool);
      for (auto& e : c->prof_ev) HIPCHK(c, hipEventCreate(&e));
      c->prof_id.resize(kProfPool);
      c->prof_bytes.resize(kProfPool);
    }
    c->prof_used = 0;
    for (auto& d : c->prof_dropped) d = 0;
  }
  c->prof_on = enable != 0;
  return GP_OK;
}

int gp_profile_read(gp_ctx* c, gp_kstat* out, int max, int* n_out) {
  if (!c || (!out && max > 0)) return GP_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ms[K_COUNT] = {0}, by[K_COUNT] = {0};
  long long cnt[K_COUNT] = {0};
  for (int s = 0; s < c->prof_used; ++s) {
    if (c->prof_id[s] < 0) continue;
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->prof_ev[2 * s], c->prof_ev[2 * s + 1]));
    ms[c->prof_id[s]] += t;
    by[c->prof_id[s]] += c->prof_bytes[s];
    cnt[c->prof_id[s]]++;
  }
  int k = 0;
  for (int id = 0; id < K_COUNT; ++id) {
    if (!cnt[id] && !c->prof_dropped[id]) continue;
    if (k < max) {
      std::memset(&out[k], 0, sizeof(gp_kstat));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kKName[id]);
      out[k].calls = cnt[id];
      out[k].dropped = c->prof_dropped[id];
      out[k].total_ms = ms[id];
      out[k].bytes = by[id];
    }
    ++k;
  }
  if (n_out) *n_out = k;
  return GP_OK;
}

}  // extern "C"

// 3-D grids: orchestration and entry points of the d = 3 solvers, built on the
// context, tables and launch helpers above
#include "gprox3d.inc"
