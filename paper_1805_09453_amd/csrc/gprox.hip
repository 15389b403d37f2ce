// libgprox: host orchestration and the C ABI declared in include/gprox.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gprox.h"
#include "gprox_fused.hpp"
#include "gprox_kernels.hpp"

using namespace gp;

namespace {

constexpr int kMinN = 64, kMaxN = 4096;
constexpr int kRedBlocks = 1024;  // partial-sum blocks of the reductions
constexpr int kMaxK = 8;

bool is_pow2_in_range(int n) { return n >= kMinN && n <= kMaxN && (n & (n - 1)) == 0; }
int ilog2i(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

struct Tables {  // per transform length N
  float2* tw32 = nullptr;
  double2* tw64 = nullptr;
  float2* dw32 = nullptr;   // exp(-i pi k / 2N)
  double2* dw64 = nullptr;
};

}  // namespace

struct gp_ctx {
  hipStream_t stream = nullptr;
  int max_ny = 0, max_nx = 0;
  Tables tab[13];            // index log2 N
  float* work = nullptr;     // [max_n] transform buffer
  float* work2 = nullptr;    // [2 max_n] EMD stored field wt (ping)
  float* work3 = nullptr;    // [2 max_n] EMD stored field wt (pong)
  double* work64 = nullptr;  // [2 max_n] FP64 set-up buffers
  double* partials = nullptr;
  double* result = nullptr;  // [kMaxK] finalized reductions (device)
  double* host_result = nullptr;  // pinned
  // eigenvalue tables of -Delta along each axis for the current (n, h)
  float *mux32 = nullptr, *muy32 = nullptr;
  double *mux64 = nullptr, *muy64 = nullptr;
  double *mu_host = nullptr;  // pinned staging [2 * kMaxN]
  float *mu_host32 = nullptr;
  int mu_ny = -1, mu_nx = -1;
  double mu_h = -1.0;
  // solver arena (grow-only)
  float* arena = nullptr;
  size_t arena_floats = 0;
  // per-kernel timing (gp_profile)
  bool prof_on = false;
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
  K_EMD_A, K_EMD_B, K_EMD_FINISH, K_DIV64, K_REDUCE, K_COUNT
};
const char* kKName[K_COUNT] = {"rows_fwd_dct2", "cols_solve", "rows_inv_dct2", "rows_fwd_dct2_f64",
                               "cols_solve_f64", "rows_inv_dct2_f64", "rof_A_prox_rhs_dct", "rof_B_idct_update",
                               "rof_finish", "emd_A_prox_rhs_dct", "emd_B_idct", "emd_finish", "div_f64",
                               "reduce"};
constexpr int kProfPool = 16384;

// records a start event for a launch of kind id moving `bytes`; returns the slot or -1
int prof_begin(gp_ctx* c, int id, double bytes) {
  if (!c->prof_on) return -1;
  if (c->prof_used >= kProfPool) {
    c->prof_dropped[id]++;
    return -1;
  }
  const int s = c->prof_used++;
  c->prof_id[s] = id;
  c->prof_bytes[s] = bytes;
  (void)hipEventRecord(c->prof_ev[2 * s], c->stream);
  return s;
}
void prof_end(gp_ctx* c, int s) {
  if (s >= 0) (void)hipEventRecord(c->prof_ev[2 * s + 1], c->stream);
}

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

int total_tw(int n) {
  switch (n) {
    case 64: return Sched<64>::total_tw();
    case 128: return Sched<128>::total_tw();
    case 256: return Sched<256>::total_tw();
    case 512: return Sched<512>::total_tw();
    case 1024: return Sched<1024>::total_tw();
    case 2048: return Sched<2048>::total_tw();
    case 4096: return Sched<4096>::total_tw();
  }
  return 0;
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

// eigenvalues of -Delta along each axis: (4/h^2) sin^2(pi k / 2n)
int set_mu(gp_ctx* c, int ny, int nx, double h) {
  if (c->mu_ny == ny && c->mu_nx == nx && c->mu_h == h) return GP_OK;
  // the staging buffer is reused: wait for any pending upload to finish
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double* hy = c->mu_host;
  double* hx = c->mu_host + kMaxN;
  float* fy = c->mu_host32;
  float* fx = c->mu_host32 + kMaxN;
  for (int k = 0; k < ny; ++k) {
    const double s = sin(M_PI * k / (2.0 * ny));
    hy[k] = 4.0 / (h * h) * s * s;
    fy[k] = float(hy[k]);
  }
  for (int l = 0; l < nx; ++l) {
    const double s = sin(M_PI * l / (2.0 * nx));
    hx[l] = 4.0 / (h * h) * s * s;
    fx[l] = float(hx[l]);
  }
  HIPCHK(c, hipMemcpyAsync(c->muy64, hy, ny * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mux64, hx, nx * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->muy32, fy, ny * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->mux32, fx, nx * sizeof(float), hipMemcpyHostToDevice, c->stream));
  c->mu_ny = ny;
  c->mu_nx = nx;
  c->mu_h = h;
  return GP_OK;
}

// ---------------------------------------------------------------- DCT launchers
// log2 of the strip width of the tiled intermediate, fixed by the column pass over ny
template <class C> int col_lgtw(int ny) {
  switch (ny) {
#define GP_TW(NN) case NN: return ilog2i(2 * ColShape<NN, C>::G);
    GP_TW(64) GP_TW(128) GP_TW(256) GP_TW(512) GP_TW(1024) GP_TW(2048) GP_TW(4096)
#undef GP_TW
  }
  return 0;
}

template <int N, class C> void launch_rows_fwd(gp_ctx* c, const typename Cx<C>::R* in, typename Cx<C>::R* out,
                                               int ny, const C* tw, const C* dw) {
  using SH = RowShape<N, C>;
  const int pairs = (ny + 1) / 2;
  const int blocks = (pairs + SH::G - 1) / SH::G;
  hipLaunchKernelGGL((k_rows_fwd<N, C>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, in, out, ny,
                     col_lgtw<C>(ny), tw, dw);
}
template <int N, class C> void launch_rows_inv(gp_ctx* c, const typename Cx<C>::R* in, typename Cx<C>::R* out,
                                               int ny, const C* tw, const C* dw) {
  using SH = RowShape<N, C>;
  const int pairs = (ny + 1) / 2;
  const int blocks = (pairs + SH::G - 1) / SH::G;
  hipLaunchKernelGGL((k_rows_inv<N, C>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, in, out, ny,
                     col_lgtw<C>(ny), tw, dw);
}
template <int N, class C> void launch_cols(gp_ctx* c, typename Cx<C>::R* buf, int nx, const C* tw, const C* dw,
                                           const typename Cx<C>::R* mux, const typename Cx<C>::R* muy,
                                           typename Cx<C>::R alpha, typename Cx<C>::R inv_nn) {
  using SH = ColShape<N, C>;
  const int pairs = nx / 2;
  const int blocks = (pairs + SH::G - 1) / SH::G;
  hipLaunchKernelGGL((k_cols_solve<N, C>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, buf, nx, tw,
                     dw, mux, muy, alpha, inv_nn);
}

template <class C> const C* tw_of(const Tables& T);
template <> const float2* tw_of<float2>(const Tables& T) { return T.tw32; }
template <> const double2* tw_of<double2>(const Tables& T) { return T.tw64; }
template <class C> const C* dw_of(const Tables& T);
template <> const float2* dw_of<float2>(const Tables& T) { return T.dw32; }
template <> const double2* dw_of<double2>(const Tables& T) { return T.dw64; }

#define GP_DISPATCH_NM(n, T, M, ...)             \
  switch (n) {                                   \
    case 64: T<64>::M(__VA_ARGS__); break;       \
    case 128: T<128>::M(__VA_ARGS__); break;     \
    case 256: T<256>::M(__VA_ARGS__); break;     \
    case 512: T<512>::M(__VA_ARGS__); break;     \
    case 1024: T<1024>::M(__VA_ARGS__); break;   \
    case 2048: T<2048>::M(__VA_ARGS__); break;   \
    case 4096: T<4096>::M(__VA_ARGS__); break;   \
  }

#define GP_DISPATCH_N(n, F, ...)            \
  switch (n) {                              \
    case 64: F<64>(__VA_ARGS__); break;     \
    case 128: F<128>(__VA_ARGS__); break;   \
    case 256: F<256>(__VA_ARGS__); break;   \
    case 512: F<512>(__VA_ARGS__); break;   \
    case 1024: F<1024>(__VA_ARGS__); break; \
    case 2048: F<2048>(__VA_ARGS__); break; \
    case 4096: F<4096>(__VA_ARGS__); break; \
  }

template <class C> struct Solve {
  using Re = typename Cx<C>::R;
  template <int N> static void rows_fwd(gp_ctx* c, const Re* in, Re* out, int ny) {
    const Tables& T = c->tab[ilog2i(N)];
    launch_rows_fwd<N, C>(c, in, out, ny, tw_of<C>(T), dw_of<C>(T));
  }
  template <int N> static void rows_inv(gp_ctx* c, const Re* in, Re* out, int ny) {
    const Tables& T = c->tab[ilog2i(N)];
    launch_rows_inv<N, C>(c, in, out, ny, tw_of<C>(T), dw_of<C>(T));
  }
  template <int N> static void cols(gp_ctx* c, Re* buf, int nx, const Re* mux, const Re* muy, Re alpha, Re inv_nn) {
    const Tables& T = c->tab[ilog2i(N)];
    launch_cols<N, C>(c, buf, nx, tw_of<C>(T), dw_of<C>(T), mux, muy, alpha, inv_nn);
  }
};

// (alpha I - Delta) x = b on the device, b and x may alias.  Tables and mu must be set.
// (alpha I - Delta) x = b: row DCT into the tiled intermediate tmp, column solve,
// row inverse into x.  b and x may alias; tmp must not alias either.
int poisson_f32(gp_ctx* c, const float* b, float* x, int ny, int nx, double alpha, float* tmp) {
  const double fb = 8.0 * double(nx) * ny;  // each pass reads and writes one FP32 field
  int ps = prof_begin(c, K_ROWS_FWD, fb);
  GP_DISPATCH_N(nx, Solve<float2>::rows_fwd, c, b, tmp, ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_COLS, fb);
  GP_DISPATCH_N(ny, Solve<float2>::cols, c, tmp, nx, c->mux32, c->muy32, float(alpha), float(1.0 / (double(nx) * ny)));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROWS_INV, fb);
  GP_DISPATCH_N(nx, Solve<float2>::rows_inv, c, tmp, x, ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}
int poisson_f64(gp_ctx* c, const double* b, double* x, int ny, int nx, double alpha, double* tmp) {
  const double fb = 16.0 * double(nx) * ny;
  int ps = prof_begin(c, K_ROWS_FWD64, fb);
  GP_DISPATCH_N(nx, Solve<double2>::rows_fwd, c, b, tmp, ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_COLS64, fb);
  GP_DISPATCH_N(ny, Solve<double2>::cols, c, tmp, nx, c->mux64, c->muy64, alpha, 1.0 / (double(nx) * ny));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROWS_INV64, fb);
  GP_DISPATCH_N(nx, Solve<double2>::rows_inv, c, tmp, x, ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

int prepare(gp_ctx* c, int ny, int nx, double h) {
  if (!is_pow2_in_range(ny) || !is_pow2_in_range(nx)) {
    set_err(c, "grid %dx%d unsupported: sides must be powers of two in [%d, %d]", ny, nx, kMinN, kMaxN);
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
  int rc = build_tables(c, ny);
  if (rc) return rc;
  rc = build_tables(c, nx);
  if (rc) return rc;
  return set_mu(c, ny, nx, h);
}

// reductions: finalize K partial columns from nb blocks into c->result and copy to host (sync)
int finalize_read(gp_ctx* c, int nb, int K, unsigned max_mask, double* out) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->stream, c->partials, nb, K, max_mask, c->result);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < K; ++i) out[i] = c->host_result[i];
  return GP_OK;
}

int count_nonfinite(gp_ctx* c, const float* x, size_t n, double* cnt) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_nonfinite, dim3(nb), dim3(256), 0, c->stream, x, n, c->partials);
  LAUNCHCHK(c);
  return finalize_read(c, nb, 1, 0u, cnt);
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

// ---------------------------------------------------------------- fused iterations
template <int N> struct Fused {
  static void rof_A(gp_ctx* c, const float* u, const float* pin, float* pout, const float* I, float* rhat, int ny,
                    float lt, float tau_h, float sig_h, int aniso, int mode, double* partials) {
    using SH = RowShape<N, float2>;
    const int blocks = (ny / 2 + SH::G - 1) / SH::G;
    const Tables& T = c->tab[ilog2i(N)];
    hipLaunchKernelGGL((k_rof_A<N>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, u, pin, pout, I,
                       rhat, ny, col_lgtw<float2>(ny), lt, tau_h, sig_h, aniso, mode, partials, T.tw32, T.dw32);
  }
  static void rof_B(gp_ctx* c, const float* dhat, float* u, int ny) {
    using SH = RowShape<N, float2>;
    const int blocks = (ny / 2 + SH::G - 1) / SH::G;
    const Tables& T = c->tab[ilog2i(N)];
    hipLaunchKernelGGL((k_rof_B<N>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, dhat, u, ny,
                       col_lgtw<float2>(ny), T.tw32, T.dw32);
  }
  static void emd_A(gp_ctx* c, const float* wt_in, const double* phi, const float* pin, const float* gpsi,
                    const float* f, float* pout, float* wt_out, double* rhat, int ny, double inv_h, float tau,
                    float sigma, int aniso, int mode, double* partials) {
    using SH = RowShape<N, double2>;
    const int blocks = (ny / 2 + SH::G - 1) / SH::G;
    const Tables& T = c->tab[ilog2i(N)];
    hipLaunchKernelGGL((k_emd_A<N>), dim3(blocks), dim3(SH::THREADS), SH::LDS_BYTES, c->stream, wt_in, phi, pin,
                       gpsi, f, pout, wt_out, rhat, ny, col_lgtw<double2>(ny), inv_h, tau, sigma, aniso, mode, partials,
                       T.tw64, T.dw64);
  }
};

int rows_blocks_f32(int nx, int ny) {
  switch (nx) {
#define GP_RB(NN) case NN: return (ny / 2 + RowShape<NN, float2>::G - 1) / RowShape<NN, float2>::G;
    GP_RB(64) GP_RB(128) GP_RB(256) GP_RB(512) GP_RB(1024) GP_RB(2048) GP_RB(4096)
#undef GP_RB
  }
  return 0;
}
int rows_blocks_f64(int nx, int ny) {
  switch (nx) {
#define GP_RB(NN) case NN: return (ny / 2 + RowShape<NN, double2>::G - 1) / RowShape<NN, double2>::G;
    GP_RB(64) GP_RB(128) GP_RB(256) GP_RB(512) GP_RB(1024) GP_RB(2048) GP_RB(4096)
#undef GP_RB
  }
  return 0;
}

// ROF pipeline.  A(entry) builds rhat from (u_n, pbar_n); each later A advances the
// dual (p ping-pong between the two state buffers) and builds the next rhat.
struct RofPipe {
  gp_ctx* c;
  const gp_state* s;
  float* X;  // buffer holding the latest complete dual iterate
  float* Y;  // the other dual buffer
  size_t n;
  float lt, tau_h, sig_h;
};

int rof_A(RofPipe& P, int mode, double* partials) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  const double by = (mode == 1 ? 20.0 : 28.0) * double(P.n);
  const int ps = prof_begin(c, K_ROF_A, by);
  const float* pin = (mode == 1) ? s->pbar : P.X;
  GP_DISPATCH_NM(s->nx, Fused, rof_A, c, s->u, pin, P.Y, s->f, c->work, s->ny, P.lt, P.tau_h, P.sig_h, s->norm,
                mode, partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  if (mode == 0) std::swap(P.X, P.Y);
  return GP_OK;
}

int rof_CB(RofPipe& P) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  const double fb = 8.0 * double(P.n);
  int ps = prof_begin(c, K_COLS, fb);
  GP_DISPATCH_N(s->ny, Solve<float2>::cols, c, c->work, s->nx, c->mux32, c->muy32, float(s->lambda * s->tau),
                float(1.0 / double(P.n)));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_ROF_B, 12.0 * double(P.n));
  GP_DISPATCH_NM(s->nx, Fused, rof_B, c, c->work, s->u, s->ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

int rof_finish(RofPipe& P) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  const int ps = prof_begin(c, K_ROF_FINISH, 28.0 * double(P.n));
  hipLaunchKernelGGL(k_rof_finish, dim3(grid_for(P.n)), dim3(256), 0, c->stream, s->u, P.X, s->p, s->pbar, s->ny,
                     s->nx, P.sig_h, s->norm);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

RofPipe rof_pipe(gp_ctx* c, const gp_state* s) {
  RofPipe P{c, s, s->p, s->pbar, size_t(s->ny) * s->nx, float(s->lambda * s->tau), float(s->tau / s->h),
            float(s->sigma / s->h)};
  return P;
}

// advance (u_n, p_n, pbar_n) by k >= 1 iterations
int rof_advance(gp_ctx* c, const gp_state* s, int k) {
  RofPipe P = rof_pipe(c, s);
  int rc = rof_A(P, 1, nullptr);
  for (int i = 0; !rc && i < k; ++i) {
    rc = rof_CB(P);
    if (!rc && i + 1 < k) rc = rof_A(P, 0, nullptr);
  }
  if (!rc) rc = rof_finish(P);
  return rc;
}

// EMD pipeline: wt ping-pong in work2/work3, phi in work64[0, n), rhat in work64[n, 2n).
struct EmdPipe {
  gp_ctx* c;
  const gp_state* s;
  float *X, *Y;    // dual buffers
  float *WX, *WY;  // wt buffers (WX = latest)
  double *phi, *rhat;
  size_t n;
};

EmdPipe emd_pipe(gp_ctx* c, const gp_state* s) {
  const size_t n = size_t(s->ny) * s->nx;
  EmdPipe P{c, s, s->p, s->pbar, c->work3, c->work2, c->work64, c->work64 + n, n};
  return P;
}

int emd_A(EmdPipe& P, int mode, double* partials) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  const double by = (mode == 1 ? 44.0 : 52.0) * double(P.n);
  const int ps = prof_begin(c, K_EMD_A, by);
  const float* win = (mode == 1) ? s->u : P.WX;
  const float* pin = (mode == 1) ? s->pbar : P.X;
  GP_DISPATCH_NM(s->nx, Fused, emd_A, c, win, P.phi, pin, s->gpsi, s->f, P.Y, P.WY, P.rhat, s->ny, 1.0 / s->h,
                float(s->tau), float(s->sigma), s->norm, mode, partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  std::swap(P.WX, P.WY);
  if (mode == 0) std::swap(P.X, P.Y);
  return GP_OK;
}

int emd_CB(EmdPipe& P) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  int ps = prof_begin(c, K_COLS64, 16.0 * double(P.n));
  GP_DISPATCH_N(s->ny, Solve<double2>::cols, c, P.rhat, s->nx, c->mux64, c->muy64, 0.0, 1.0 / double(P.n));
  prof_end(c, ps);
  LAUNCHCHK(c);
  ps = prof_begin(c, K_EMD_B, 16.0 * double(P.n));
  GP_DISPATCH_N(s->nx, Solve<double2>::rows_inv, c, P.rhat, P.phi, s->ny);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

// write (u, p, pbar) of the state from (wt, phi, latest p); m and partials optional
int emd_finish(EmdPipe& P, float* m, double* partials, int nb) {
  gp_ctx* c = P.c;
  const gp_state* s = P.s;
  const int ps = prof_begin(c, K_EMD_FINISH, 56.0 * double(P.n));
  hipLaunchKernelGGL(k_emd_finish, dim3(nb), dim3(256), 0, c->stream, P.WX, P.phi, P.X, s->gpsi, s->p, s->pbar,
                     s->u, m, s->ny, s->nx, 1.0 / s->h, float(s->sigma), s->norm, partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  return GP_OK;
}

int emd_advance(gp_ctx* c, const gp_state* s, int k) {
  EmdPipe P = emd_pipe(c, s);
  int rc = emd_A(P, 1, nullptr);
  for (int i = 0; !rc && i < k; ++i) {
    rc = emd_CB(P);
    if (!rc && i + 1 < k) rc = emd_A(P, 0, nullptr);
  }
  if (!rc) rc = emd_finish(P, nullptr, nullptr, grid_for(P.n));
  return rc;
}

int rof_gap(gp_ctx* c, const gp_state* s, double* P, double* D) {
  const size_t n = size_t(s->ny) * s->nx;
  const int nb = red_blocks(n);
  int ps = prof_begin(c, K_REDUCE, 16.0 * n);
  hipLaunchKernelGGL(k_rof_energy, dim3(nb), dim3(256), 0, c->stream, s->u, s->p, s->p + n, s->f, s->ny, s->nx,
                     float(1.0 / s->h), s->norm, c->partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  double r[4];
  int rc = finalize_read(c, nb, 4, 0u, r);
  if (rc) return rc;
  const double h2 = s->h * s->h;
  *P = h2 * (r[0] + 0.5 * s->lambda * r[1]);
  *D = -h2 * (r[2] + r[3] / (2.0 * s->lambda));
  return GP_OK;
}

// certificate D from p: phi = Delta^{-1} div p, D = -h^2 sum phi f / max(1, max|grad phi|).
// Leaves -phi (FP64) in c->work64; *L receives max|grad phi|.
int emd_cert(gp_ctx* c, const gp_state* s, double* D, double* L, double* phi, double* tmp) {
  const size_t n = size_t(s->ny) * s->nx;
  int ps = prof_begin(c, K_DIV64, 16.0 * n);
  hipLaunchKernelGGL(k_div<double>, dim3(grid_for(n)), dim3(256), 0, c->stream, s->p, s->p + n, phi, s->ny, s->nx,
                     float(1.0 / s->h));
  prof_end(c, ps);
  LAUNCHCHK(c);
  // Delta phi = div p  <=>  (0 I - Delta) phi = -div p: this solves for -phi; the sign is
  // folded into D below
  int rc = poisson_f64(c, phi, phi, s->ny, s->nx, 0.0, tmp);
  if (rc) return rc;
  const int nb = red_blocks(n);
  ps = prof_begin(c, K_REDUCE, 12.0 * n);
  hipLaunchKernelGGL(k_emd_cert, dim3(nb), dim3(256), 0, c->stream, phi, s->f, s->ny, s->nx, 1.0 / s->h, s->norm,
                     c->partials);
  prof_end(c, ps);
  LAUNCHCHK(c);
  double r[2];
  rc = finalize_read(c, nb, 2, 2u, r);
  if (rc) return rc;
  // phi holds -phi_c; sum(-phi_c f) = r[0]
  *L = r[1];
  *D = s->h * s->h * r[0] / (r[1] > 1.0 ? r[1] : 1.0);
  return GP_OK;
}

int emd_primal(gp_ctx* c, const gp_state* s, double* P) {
  const size_t n = size_t(s->ny) * s->nx;
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_emd_primal, dim3(nb), dim3(256), 0, c->stream, s->u, s->u + n, s->gpsi, s->gpsi + n, n,
                     s->norm, c->partials);
  LAUNCHCHK(c);
  double r[1];
  int rc = finalize_read(c, nb, 1, 0u, r);
  if (rc) return rc;
  *P = s->h * s->h * r[0];
  return GP_OK;
}

double rel_gap(double P, double D) { return P != 0.0 ? (P - D) / fabs(P) : fabs(P - D); }

int validate_state(gp_ctx* c, const gp_state* s) {
  if (!s || !s->f || !s->u || !s->p || !s->pbar || (s->kind == GP_KIND_EMD && !s->gpsi)) {
    set_err(c, "state has a NULL buffer");
    return GP_EINVAL;
  }
  if (s->kind != GP_KIND_ROF && s->kind != GP_KIND_EMD) {
    set_err(c, "state kind must be GP_KIND_ROF or GP_KIND_EMD");
    return GP_EINVAL;
  }
  if (!(s->tau > 0) || !(s->sigma > 0) || s->tau * s->sigma > 1.0 + 1e-12 ||
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

const char* gp_last_error(const gp_ctx* ctx) { return ctx ? ctx->err : "no context"; }

int gp_create(gp_ctx** out, int max_ny, int max_nx, void* stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  if (!is_pow2_in_range(max_ny) || !is_pow2_in_range(max_nx)) return GP_EUNSUPPORTED;
  gp_ctx* c = new (std::nothrow) gp_ctx();
  if (!c) return GP_ENOMEM;
  c->stream = static_cast<hipStream_t>(stream);
  c->max_ny = max_ny;
  c->max_nx = max_nx;
  const size_t n = size_t(max_ny) * max_nx;
  bool ok = hipMalloc(&c->work, n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work2, 2 * n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work3, 2 * n * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->work64, 2 * n * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->partials, size_t(kRedBlocks) * kMaxK * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->result, kMaxK * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&c->host_result, kMaxK * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->mux32, kMaxN * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->muy32, kMaxN * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->mux64, kMaxN * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->muy64, kMaxN * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&c->mu_host, 2 * kMaxN * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&c->mu_host32, 2 * kMaxN * sizeof(float)) == hipSuccess;
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
  if (c->stream) (void)hipStreamSynchronize(c->stream);
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
  for (auto& e : c->prof_ev) (void)hipEventDestroy(e);
  if (c->host_result) (void)hipHostFree(c->host_result);
  if (c->mu_host) (void)hipHostFree(c->mu_host);
  if (c->mu_host32) (void)hipHostFree(c->mu_host32);
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
  int rc = prepare(c, ny, nx, h);
  if (rc) return rc;
  return poisson_f32(c, b, x, ny, nx, alpha, c->work);
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
  int rc = prepare(c, ny, nx, h);
  if (rc) return rc;
  return poisson_f64(c, b, x, ny, nx, alpha, c->work64);
}

int pd_step(gp_ctx* c, gp_state* s, int n_iter) {
  if (!c) return GP_EINVAL;
  if (n_iter < 0) {
    set_err(c, "n_iter < 0");
    return GP_EINVAL;
  }
  int rc = validate_state(c, s);
  if (rc || n_iter == 0) return rc;
  rc = (s->kind == GP_KIND_ROF) ? rof_advance(c, s, n_iter) : emd_advance(c, s, n_iter);
  if (rc) return rc;
  s->iter += n_iter;
  return GP_OK;
}

int pd_gap(gp_ctx* c, gp_state* s, gp_report* rep) {
  if (!c) return GP_EINVAL;
  int rc = validate_state(c, s);
  if (rc) return rc;
  double P = 0, D = 0, L = 0;
  if (s->kind == GP_KIND_ROF) {
    rc = rof_gap(c, s, &P, &D);
  } else {
    rc = emd_primal(c, s, &P);
    if (!rc) rc = emd_cert(c, s, &D, &L, c->work64, c->work64 + size_t(s->ny) * s->nx);
  }
  if (rc) return rc;
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
  int rc = check_opts(c, o, &tau, &sigma);
  if (rc) return rc;
  rc = prepare(c, ny, nx, h);
  if (rc) return rc;
  const size_t n = size_t(ny) * nx;
  double bad = 0;
  rc = count_nonfinite(c, I, n, &bad);
  if (rc) return rc;
  if (bad > 0) {
    set_err(c, "image has %.0f non-finite values", bad);
    return GP_EINVAL;
  }
  float* ar = arena(c, 4 * n);
  if (!ar) {
    set_err(c, "arena allocation of %zu floats failed", 4 * n);
    return GP_ENOMEM;
  }
  // dual buffers: P0 holds p_0 (and the final p), P1 holds pbar_0
  float* P0 = ar;
  float* P1 = ar + 2 * n;
  if (o->warm_start && p) {
    HIPCHK(c, hipMemcpyAsync(P0, p, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  } else {
    HIPCHK(c, hipMemsetAsync(P0, 0, 2 * n * sizeof(float), c->stream));
  }
  if (!o->warm_start) HIPCHK(c, hipMemsetAsync(u, 0, n * sizeof(float), c->stream));
  HIPCHK(c, hipMemcpyAsync(P1, P0, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  gp_state s{GP_KIND_ROF, ny, nx, o->norm, h, lambda, tau, sigma, I, nullptr, u, P0, P1, 0};
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t1 = now_s();
  double P = NAN, D = NAN, g = NAN;
  bool conv = false;
  int it = 0;
  RofPipe pipe = rof_pipe(c, &s);
  rc = rof_A(pipe, 1, nullptr);
  if (rc) return rc;
  const int nb = rows_blocks_f32(nx, ny);
  while (it < o->max_iter) {
    rc = rof_CB(pipe);  // u_{it+1}
    if (rc) return rc;
    ++it;
    const bool chk = (it % o->check_every == 0) || (it == o->max_iter);
    // A computes p_it from (u_it, p_{it-1}) and, on checks, the gap of (u_it, p_it)
    rc = rof_A(pipe, 0, chk ? c->partials : nullptr);
    if (rc) return rc;
    if (chk) {
      double r[4];
      rc = finalize_read(c, nb, 4, 0u, r);
      if (rc) return rc;
      P = h * r[0] + 0.5 * lambda * h * h * r[1];
      D = -h * r[2] - r[3] / (2.0 * lambda);
      g = rel_gap(P, D);
      if (!std::isfinite(g)) {
        set_err(c, "duality gap became non-finite at iteration %d", it);
        return GP_EHIP;
      }
      if (g <= o->tol) {
        conv = true;
        break;
      }
    }
  }
  if (p) HIPCHK(c, hipMemcpyAsync(p, pipe.X, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t2 = now_s();
  if (rep) {
    rep->iters = it;
    rep->converged = conv;
    rep->primal = P;
    rep->dual = D;
    rep->rel_gap = g;
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
  int rc = prepare(c, ny, nx, h);
  if (rc) return rc;
  const size_t n = size_t(ny) * nx;
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(k_mass, dim3(nb), dim3(256), 0, c->stream, rho0, rho1, n, c->partials);
  LAUNCHCHK(c);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->stream, c->partials, nb, 3, 0u, c->result);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(c->host_result, c->result, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double m0 = c->host_result[0], m1 = c->host_result[1], bad = c->host_result[2];
  if (bad > 0) {
    set_err(c, "densities have %.0f negative or non-finite values", bad);
    return GP_EINVAL;
  }
  if (fabs(m0 - m1) > 1e-6 * fabs(m0)) {
    set_err(c, "mass mismatch: sum rho0 = %.17g, sum rho1 = %.17g", m0, m1);
    return GP_EMASS;
  }
  double* f64 = c->work64;
  double* psi = c->work64;  // the solve consumes f64 before writing psi over it
  double* tmp = c->work64 + n;
  hipLaunchKernelGGL(k_f64_diff, dim3(grid_for(n)), dim3(256), 0, c->stream, rho0, rho1, c->result,
                     1.0 / double(n), n, f64, f);
  LAUNCHCHK(c);
  rc = poisson_f64(c, f64, psi, ny, nx, 0.0, tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_grad_f64, dim3(grid_for(n)), dim3(256), 0, c->stream, psi, gpsi, gpsi + n, ny, nx, 1.0 / h);
  LAUNCHCHK(c);
  return GP_OK;
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
  int rc = check_opts(c, o, &tau, &sigma);
  if (rc) return rc;
  if (o->warm_start && !phi) {
    set_err(c, "warm_start needs phi");
    return GP_EINVAL;
  }
  rc = prepare(c, ny, nx, h);
  if (rc) return rc;
  const size_t n = size_t(ny) * nx;
  // arena: f, grad psi, u, P0, P1, certificate potential and its transform intermediate (n doubles each)
  float* ar = arena(c, 13 * n);
  if (!ar) {
    set_err(c, "arena allocation of %zu floats failed", 13 * n);
    return GP_ENOMEM;
  }
  float* f = ar;
  float* gpsi = ar + n;
  float* u = ar + 3 * n;
  float* P0 = ar + 5 * n;
  float* P1 = ar + 7 * n;
  double* cphi = reinterpret_cast<double*>(ar + 9 * n);
  double* ctmp = reinterpret_cast<double*>(ar + 11 * n);
  rc = emd_setup(c, rho0, rho1, f, gpsi, ny, nx, h);
  if (rc) return rc;
  HIPCHK(c, hipMemsetAsync(u, 0, 2 * n * sizeof(float), c->stream));
  HIPCHK(c, hipMemsetAsync(P0, 0, 2 * n * sizeof(float), c->stream));
  if (o->warm_start) {
    // p0 = proj(grad phi0): the ROF dual step with u = phi0, p = 0, sigma/h = 1/h
    hipLaunchKernelGGL(k_rof_finish, dim3(grid_for(n)), dim3(256), 0, c->stream, phi, P0, P0, P1, ny, nx,
                       float(1.0 / h), o->norm);
    LAUNCHCHK(c);
  }
  HIPCHK(c, hipMemcpyAsync(P1, P0, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  gp_state s{GP_KIND_EMD, ny, nx, o->norm, h, 0.0, tau, sigma, f, gpsi, u, P0, P1, 0};
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t1 = now_s();
  double P = NAN, D = NAN, g = NAN, L = 0;
  bool conv = false;
  int it = 0;
  EmdPipe pipe = emd_pipe(c, &s);
  rc = emd_A(pipe, 1, nullptr);
  if (rc) return rc;
  const int nb = rows_blocks_f64(nx, ny);
  while (it < o->max_iter) {
    rc = emd_CB(pipe);  // phi_it
    if (rc) return rc;
    const bool chk = ((it + 1) % o->check_every == 0) || (it + 1 == o->max_iter);
    rc = emd_A(pipe, 0, chk ? c->partials : nullptr);  // u_{it+1}, p_{it+1}
    if (rc) return rc;
    ++it;
    if (chk) {
      double r[1];
      rc = finalize_read(c, nb, 1, 0u, r);
      if (rc) return rc;
      P = h * h * r[0];
      gp_state cs = s;
      cs.p = pipe.X;
      rc = emd_cert(c, &cs, &D, &L, cphi, ctmp);
      if (rc) return rc;
      g = rel_gap(P, D);
      if (!std::isfinite(g)) {
        set_err(c, "duality gap became non-finite at iteration %d", it);
        return GP_EHIP;
      }
      if (g <= o->tol) {
        conv = true;
        break;
      }
    }
  }
  // flux m_it = wt_{it-1} - grad phi_{it-1} (the A that produced p_it read these)
  hipLaunchKernelGGL(k_emd_finish, dim3(grid_for(n)), dim3(256), 0, c->stream, pipe.WY, pipe.phi, nullptr, gpsi,
                     nullptr, nullptr, nullptr, m, ny, nx, 1.0 / h, float(sigma), o->norm, nullptr);
  LAUNCHCHK(c);
  if (phi) {
    // cphi holds -phi_c from the last certificate; phi~ = phi_c / max(1, L)
    hipLaunchKernelGGL(k_scale<double>, dim3(grid_for(n)), dim3(256), 0, c->stream, cphi, phi, n,
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
    rep->rel_gap = g;
    rep->div_residual = 0;
    rep->seconds_setup = t1 - t0;
    rep->seconds_loop = t2 - t1;
  }
  return conv ? GP_OK : GP_ENOTCONV;
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
