/* gprox.h - C ABI of libgprox: G-prox PDHG on 2-D grids for MI355X (gfx950).
 *
 * Method: Jacobs, Leger, Li, Osher, "Solving large-scale optimization problems
 * with a convergence rate independent of grid size" (arXiv 1805.09453):
 * Algorithm 2 (G-prox PDHG) applied to
 *   - ROF total-variation denoising (section 3.1):
 *       min_u ||u||_TV + lambda/2 ||u - I||^2,
 *   - the L1 earth mover's distance in Beckmann form (section 3.2):
 *       EMD(rho1, rho0) = min { int |m| : div m = rho1 - rho0, m.n = 0 }.
 *
 * Grid and operators.  ny x nx cell-centred grid with spacing h (the paper's
 * unit square is h = 1/n; h = 1 gives per-pixel units).  Scalar fields are
 * row-major float[ny][nx]; vector fields are planar float[2][ny][nx] (x
 * component first).  grad is the forward difference with zero normal
 * component on the far faces, div = -grad^T, Delta = div grad (Neumann), and
 * the pointwise norm is Euclidean (norm = 0) or l1 (norm = 1).  The Laplace
 * inversions (the u-step of Algorithm 2 in both problems) run as
 * DCT-II -> diagonal scale -> inverse DCT-II (section 4, appendix A).
 *
 * Memory and ownership.  Every float pointer argument is a DEVICE pointer
 * (hipMalloc'd or a torch tensor's data_ptr) to contiguous memory owned by
 * the caller; the library keeps no pointer after a call returns.  All work is
 * enqueued on the context's stream.  The library owns only the workspace in
 * its context, sized at gp_create for grids up to max_ny x max_nx (solve
 * calls may grow it; pd_step and pd_gap allocate nothing on power-of-two
 * grids, see pd_step for the other sides).
 *
 * Sizes.  ny and nx must lie in [64, 4096] with no prime factor above 7
 * (7-smooth: 64, 72, 75, 80, 81, 84, 90, 96, ... 720, ... 4096) and at most the
 * context's maxima; other sizes return GP_EUNSUPPORTED.  Powers of two run the
 * fused register-resident transforms; other sides run the same iteration
 * unfused, with mixed-radix (2, 3, 4, 5, 7, 8) DCTs out of LDS, the column
 * pass reading the columns in place (gp_opts.ergodic, the 3-D calls,
 * dct_poisson_noalloc, the launch-shape calls and the learned warm start need
 * powers of two).
 *
 * Errors.  Every entry point returns GP_OK (0), a negative GP_E* code, or
 * GP_ENOTCONV (> 0: max_iter reached, outputs valid, report filled).  No C++
 * exception crosses this boundary.  gp_last_error() gives a message for the
 * last failure on a context.
 */
#ifndef GPROX_H
#define GPROX_H

#ifdef __cplusplus
extern "C" {
#endif

#define GP_OK 0
#define GP_ENOTCONV 1       /* max_iter reached before tol; outputs valid */
#define GP_EINVAL (-1)      /* null pointer, bad size/step/h/lambda, NaN/Inf or negative input */
#define GP_EMASS (-2)       /* |sum rho0 - sum rho1| > 1e-6 sum rho0 (FP64) */
#define GP_ENOMEM (-3)      /* device allocation failed */
#define GP_EHIP (-4)        /* HIP runtime error (see gp_last_error) */
#define GP_EUNSUPPORTED (-5)/* grid size or option not supported */

#define GP_KIND_ROF 0
#define GP_KIND_EMD 1
#define GP_NORM_ISO 0
#define GP_NORM_ANISO 1

typedef struct gp_ctx gp_ctx; /* opaque: stream, twiddle tables, workspace */

/* Step sizes and stopping rule of Algorithm 2.
 * tau, sigma: primal / dual steps; sigma <= 0 selects sigma = 1/tau, the
 *   choice of every step rule in the paper (sections 3.1, 3.2, 4).  The
 *   convergence theorem of section 3 needs tau * sigma < 1; tau * sigma <= 1
 *   is accepted (the boundary case is the Douglas-Rachford equivalent).
 * tol: stop when the relative duality gap (P - D)/|P| of the last iterate
 *   (section 4 stops on the last iterate) is <= tol; 0 runs max_iter.
 * check_every: evaluate the gap every this many iterations (>= 1).
 * norm: GP_NORM_ISO or GP_NORM_ANISO.
 * warm_start: nonzero uses the caller's u/p (ROF) or phi (EMD) as the start.
 * ergodic: nonzero evaluates the gap on, and returns, the averages
 *   u^N = (1/N) sum u_n and p^N = (1/N) sum p_n over the iterates n = 1..N of
 *   this call (the ergodic iterates that the convergence rates of section 2
 *   are stated for; EMD averages the flux m_n = u_n + grad psi).  The sums are
 *   FP64 in the context's workspace (ROF 9, EMD 10 more floats of workspace
 *   per cell) and cost one more pass over them per iteration.  rof_solve,
 *   emd_solve, rof3_solve and emd3_solve; gp_batch_solve rejects it
 *   (GP_EUNSUPPORTED).
 */
typedef struct {
  double tau, sigma, tol;
  int max_iter, check_every, norm, warm_start, ergodic;
} gp_opts;

/* Filled by the solvers and by pd_gap. primal/dual are P(u) and D(p)
 * (section 2.1 primal-dual gap); div_residual is max |div m - (rho1-rho0)|
 * of the returned EMD flux (0 for ROF). */
typedef struct {
  int iters, converged;
  double primal, dual, rel_gap, div_residual;
  double seconds_setup, seconds_loop;
} gp_report;

/* Device-resident iterate for pd_step / pd_gap (all buffers caller-owned).
 *   kind  GP_KIND_ROF: f = image I [ny][nx]; u = u_n [ny][nx].
 *         GP_KIND_EMD: f = rho1 - rho0 - mean [ny][nx]; gpsi = grad psi
 *                      [2][ny][nx] with Delta psi = f (emd_setup fills both);
 *                      u = divergence-free part u_n [2][ny][nx].
 *   p, pbar: dual iterate p_n and its extrapolation 2 p_n - p_{n-1} [2][ny][nx]
 *            (pbar = p at n = 0).
 *   tau, sigma: steps (sigma <= 0 selects 1/tau, as in gp_opts); lambda: ROF only.
 *   iter: iterations done; pd_step adds n_iter. */
typedef struct {
  int kind, ny, nx, norm;
  double h, lambda, tau, sigma;
  const float* f;
  const float* gpsi;
  float* u;
  float* p;
  float* pbar;
  long long iter;
} gp_state;

/* Context on a HIP stream (NULL = default stream).  max_ny, max_nx bound the
 * grids later calls may use.  Returns GP_OK and *ctx, or an error. */
int gp_create(gp_ctx** ctx, int max_ny, int max_nx, void* stream);
int gp_destroy(gp_ctx* ctx);
const char* gp_strerror(int code);
const char* gp_last_error(const gp_ctx* ctx); /* ctx NULL: see dct_poisson_noalloc */

/* Screened Poisson solve (alpha I - Delta) x = b with Neumann boundary (the
 * linear solve of the ROF u-update, section 3.1, with alpha = lambda tau; the
 * Laplace inversion of the Leray projection, section 3.2, with alpha = 0).
 * alpha = 0: b is projected to mean zero (mean taken in FP64) and x has mean
 * zero.  b and x are float[ny][nx] device buffers and may alias. */
int dct_poisson(gp_ctx* ctx, const float* b, float* x, int ny, int nx, double h, double alpha);
/* The same in FP64 (used for the EMD set-up potential). */
int dct_poisson_f64(gp_ctx* ctx, const double* b, double* x, int ny, int nx, double h, double alpha);

/* dct_poisson for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  No
 * context: the work is enqueued on `stream` (NULL = the null stream of the
 * current device) and the call never synchronises and never allocates (no
 * hipMalloc, hipFree, memset or host-to-device copy).  Its workspace is one
 * file-scope device array of about 4.4 MB that each GPU the library runs on
 * holds until the process ends (its address is looked up once per device).
 * Limits: sides powers of two in [64, 4096] with ny * nx <= 2^20 (1024 x 1024,
 * 512 x 2048, 256 x 4096, ...); larger grids return GP_EUNSUPPORTED.  The
 * solve, the arguments and the other errors are those of dct_poisson (launch
 * shapes are the defaults, not tuned ones); gp_last_error(NULL) gives the
 * message of the last failed call of this kind on the calling thread.  Calls
 * on one GPU share the workspace: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller; each call rewrites every table it reads, so no state carries
 * over from an earlier call. */
int dct_poisson_noalloc(const float* b, float* x, int ny, int nx, double h, double alpha, void* stream);

/* ROF denoising of I (section 3.1 updates of Algorithm 2).  u: out (and in
 * when opts->warm_start) [ny][nx]; p: nullable [2][ny][nx] dual out (and in
 * when warm_start).  Stops on opts->tol or opts->max_iter; rep may be NULL. */
int rof_solve(gp_ctx* ctx, const float* I, float* u, float* p, int ny, int nx, double h, double lambda,
              const gp_opts* opts, gp_report* rep);

/* EMD between densities rho0, rho1 >= 0 of equal mass (section 3.2 updates).
 * m: out flux u + grad psi [2][ny][nx]; phi: nullable [ny][nx]; in: warm-start
 * potential phi0 (p0 = proj(grad phi0)) when opts->warm_start, out: the
 * scaled dual potential of the certificate (|grad phi| <= 1).  rep->primal is
 * the EMD upper bound h^2 sum |m|, rep->dual the certificate's lower bound.
 * With sigma tau = 1 (the default sigma) and no averaging, the iterates are
 * formed in the equivalent single-variable form (state y = p_prev + sigma
 * (u + grad psi), p = proj(y); the Douglas-Rachford case of section 2; a
 * warm start is y0 = p0); otherwise in the two-variable form. */
int emd_solve(gp_ctx* ctx, const float* rho0, const float* rho1, float* m, float* phi, int ny, int nx, double h,
              const gp_opts* opts, gp_report* rep);

/* EMD set-up (section 3.2, Hodge split): mass check in FP64, f = rho1 - rho0
 * - mean (FP64), psi = Delta^{-1} f solved in FP64, gpsi = grad psi stored
 * FP32.  f: out [ny][nx]; gpsi: out [2][ny][nx]. */
int emd_setup(gp_ctx* ctx, const float* rho0, const float* rho1, float* f, float* gpsi, int ny, int nx,
              double h);

/* Step sizes from the data, computed before a solve.
 *
 * ROF (section 4.1): tau = min(sqrt(lambda) ||I||_TV / sqrt(eps), ||grad I||_L2),
 * sigma = 1/tau, where ||I||_TV = h^2 sum |grad I| (the pointwise norm `norm`)
 * and ||grad I||_L2 = sqrt(h^2 sum |grad I|_2^2), forward differences as the
 * solver's.  The first term alone is the grid-independent choice (section 4.1,
 * the lambda = 20 experiment without the grid cap).  tv_bound is the bound of
 * section 3.1 on the minimiser, ||u*||_TV <= min(||I||_TV, lambda/2 ||I0 - I||^2)
 * with I0 the mean of I.  eps is the absolute objective error the rule targets.
 * FP64 sums on the device from the FP32 image; synchronises the stream.
 * GP_EINVAL for NULL arguments, lambda or eps not positive and finite, a bad
 * norm or a non-finite image; sizes as rof_solve. */
typedef struct {
  double tv, grad_l2, tv_bound;
  double tau;            /* min(tau_continuum, grad_l2) */
  double tau_continuum;  /* sqrt(lambda) tv / sqrt(eps) */
} gp_rof_rule;
int rof_step_rule(gp_ctx* ctx, const float* I, int ny, int nx, double h, double lambda, double eps, int norm,
                  gp_rof_rule* out);

/* EMD rule for singular measures (section 4.2): tau = min(sqrt(1 / (eps |ln eps|)),
 * 2 m^(1/4)), sigma = 1/tau, for a grid of side m (the paper's statements about
 * which term binds on its grids hold for m the side length and the natural
 * logarithm).  Host arithmetic only; returns -1 unless 0 < eps < 1 and m > 0. */
double emd_step_rule_singular(double eps, double m);

/* Advance a device-resident iterate by n_iter G-prox PDHG iterations:
 * Algorithm 2 (u-step in the H-inner product, dual prox, extrapolation
 * pbar = 2 p_{n+1} - p_n) with the ROF updates of section 3.1 (u-step by the
 * screened Poisson solve with alpha = lambda tau, incremental form) or the EMD
 * updates of section 3.2 (u-step by the Leray projection, projected form
 * u+ = P(u - tau pbar)); the dual steps project pointwise onto |p| <= 1.
 * The state is the two-variable iterate (u_n, p_n, pbar_n) in either case.
 * On power-of-two grids it enqueues work only: never synchronises, never
 * allocates.  On other grids the iteration's launches read a small device
 * table of their arguments (the form gp_batch_solve uses, so that both compute
 * the same bits); the first call for a state, and any call after the state's
 * buffers or parameters changed, writes that table: it synchronises the
 * stream once and may allocate a few KB.  Later calls only enqueue. */
int pd_step(gp_ctx* ctx, gp_state* st, int n_iter);

/* Primal value, dual value and relative gap of the state's (u_n, p_n);
 * synchronises the stream once. */
int pd_gap(gp_ctx* ctx, gp_state* st, gp_report* rep);

/* ---- 3-D grids: the d = 3 case of section 3 (the theory of sections 2-3 is
 * stated for general d).  Grids nz x ny x nx, each side a power of two in
 * [64, 4096], at most 2^27 cells; scalar fields float[nz][ny][nx] (x
 * fastest), vector fields planar float[3][nz][ny][nx] (x, y, z components).
 * Operators: forward-difference gradient (zero on the far faces), divergence
 * its negative adjoint, the 7-point Neumann Laplacian, h^3 sums; pointwise
 * norms |p| = sqrt(px^2 + py^2 + pz^2) (GP_NORM_ISO) or |px| + |py| + |pz|
 * (GP_NORM_ANISO).  Workspace: the context's arena (grown on demand: ROF
 * about 40, EMD about 64 bytes per cell); all buffers caller-owned device
 * memory; errors as the 2-D calls (GP_EUNSUPPORTED for other sizes). */

/* (alpha I - Delta) x = b, Neumann, by the 3-D DCT-II (the linear solves of
 * sections 3.1 and 3.2 in d = 3); alpha = 0 drops the zero mode (x has mean
 * zero).  b and x may alias.  FP32 and FP64 variants. */
int dct_poisson3(gp_ctx* ctx, const float* b, float* x, int nz, int ny, int nx, double h, double alpha);
int dct_poisson3_f64(gp_ctx* ctx, const double* b, double* x, int nz, int ny, int nx, double h, double alpha);

/* ROF denoising of the volume I (section 3.1 updates in d = 3) from u = 0,
 * p = 0, or from the caller's u and p with opts->warm_start.  u: in/out
 * [nz][ny][nx]; p: nullable in/out [3][nz][ny][nx].  Gap, stopping rule and
 * report as rof_solve (P and D with h^3 sums); opts->ergodic averages as
 * rof_solve (about 44 more bytes of workspace per cell). */
int rof3_solve(gp_ctx* ctx, const float* I, float* u, float* p, int nz, int ny, int nx, double h, double lambda,
               const gp_opts* opts, gp_report* rep);

/* EMD between volumes rho0, rho1 >= 0 of equal mass (section 3.2 updates in
 * d = 3, projected form, FP64 potentials) from the zero start or a warm
 * start.  m: out flux u + grad psi [3][nz][ny][nx]; rep->primal = h^3 sum
 * |m|, rep->dual the certificate's lower bound.  phi: nullable
 * [nz][ny][nx]; in: the warm-start potential
 * phi0 when opts->warm_start (p0 = proj(grad phi0), u0 = 0, as emd_solve),
 * out: the scaled certificate potential.  opts->ergodic averages the flux
 * and p as emd_solve (about 72 more bytes per cell).
 * With sigma tau = 1 (the default sigma) and no averaging the same iterates
 * are formed in the
 * equivalent single-variable form (state y = p_prev + sigma (u + grad psi),
 * p = proj(y); the Douglas-Rachford case of section 2), which stores one
 * vector field instead of two. */
int emd3_solve(gp_ctx* ctx, const float* rho0, const float* rho1, float* m, float* phi, int nz, int ny, int nx,
               double h, const gp_opts* opts, gp_report* rep);

/* One problem of a batch.
 *   GP_KIND_ROF: in0 = image I [ny][nx]; out = u [ny][nx]; lambda > 0.
 *   GP_KIND_EMD: in0 = rho0, in1 = rho1 [ny][nx] (equal mass); out = flux m
 *                [2][ny][nx] (lambda ignored).
 * tau is the instance's primal step (sigma = 1/tau, as in every step rule of
 * sections 3.1, 3.2 and 4). */
typedef struct {
  int kind, ny, nx;
  double h, lambda, tau;
  const float* in0;
  const float* in1;
  float* out;
  float* phi; /* EMD, nullable: out [ny][nx] scaled certificate potential (as emd_solve) */
} gp_instance;

/* Solve count independent instances (each one the solve of rof_solve or
 * emd_solve from a zero start; the iteration is section 3's Algorithm 2 per
 * instance, nothing couples instances).  Instances of the same kind, size, h,
 * lambda and tau run stacked in one set of launches; one hipGraph holds a
 * chunk of iterations of every group plus their duality gaps, and is replayed
 * on a private stream of the context until every instance has met opts->tol
 * or run opts->max_iter iterations.  A converged instance retires at the
 * check where it converged: its kernels skip it from then on, so its outputs
 * equal those of the matching single-instance solve with the same
 * check_every (rounded up to even, the chunk length C; iteration counts are
 * multiples of C).  An instance that has not converged stops at the first
 * check at or after opts->max_iter, so it may run up to C - 1 iterations
 * beyond max_iter (check_every 5, max_iter 20: C = 6, 24 iterations).
 * opts->tau/sigma are ignored (per-instance tau, sigma = 1/tau: EMD instances
 * run the single-variable form as emd_solve); opts->warm_start must be 0
 * (GP_EINVAL otherwise), and so must be a non-finite ROF image or negative or
 * non-finite densities (the error names the instance).  reps: nullable array of count reports;
 * seconds_loop is the time from the first replay to the instance's last
 * check.  Allocates the batch workspace (grow-only, kept in the context) and
 * synchronises.  Returns GP_OK when every instance converged, GP_ENOTCONV
 * when some reached max_iter (all outputs valid), or an error (GP_EMASS names
 * the first instance with unequal masses in gp_last_error). */
int gp_batch_solve(gp_ctx* ctx, const gp_instance* inst, int count, const gp_opts* opts, gp_report* reps);

/* Launch shapes (a performance setting; results do not depend on it).  Each
 * DCT pass runs FFT groups of n/32 threads (n <= 128) or n/16 threads
 * (n >= 256), one per row pair (row passes) or column pair (column pass).
 * For transforms of length n in FP32 (fp64 = 0: the ROF path and dct_poisson)
 * or FP64 (fp64 = 1: the EMD path and dct_poisson_f64) these calls read or set
 *   row_groups  FFT groups per row-pass workgroup (rows of length n; in FP32
 *               the tuner measures the ROF row inverse on its own and may give
 *               it another count; gp_set_shape sets both, gp_get_shape reports
 *               the first row pass's);
 *   col_groups  FFT groups per column-pass workgroup (columns of length n);
 *   tile_width  strip width of the column-tiled intermediate between the row
 *               and column passes of columns of length n (used clamped to
 *               [2 col_groups, grid width]).
 * rof_solve, emd_solve and gp_batch_solve measure the candidates on first use
 * of a size and keep the fastest (an autotuner; pd_step and dct_poisson use
 * the current setting); gp_set_shape fixes a choice (0 leaves a setting
 * unchanged; a column setting fixes both column values) and exempts it from
 * tuning.  Row groups must fill whole 64-lane waves within the 256-thread
 * (512 for n >= 256) and LDS limits; column groups must be a power of two
 * within the LDS and 512-thread (1024 for n >= 256) limits; the tile width a
 * power of two in [2, 64]; GP_EINVAL otherwise.  Out pointers may be NULL. */
int gp_get_shape(gp_ctx* ctx, int fp64, int n, int* row_groups, int* col_groups, int* tile_width);
int gp_set_shape(gp_ctx* ctx, int fp64, int n, int row_groups, int col_groups, int tile_width);

/* Radix plan of the transforms of a side n that is 7-smooth but not a power of
 * two (appendix A: the cosine-series inversion holds for any n).  A plan lists
 * the radices of the Stockham passes in order: each 2, 3, 4, 5, 7 or 8, with
 * product n, at most 16 passes.  On the first transform of such a length in a
 * precision the library times its candidate plans (the odd radices first or
 * last, the power-of-two factor as radix-8 or radix-4 passes) and keeps the
 * fastest; the default (odd radices first, radix-8 passes) unless another is at
 * least 3% faster.  Every plan computes the same DCT; only rounding differs.
 * Nothing is measured on a stream under graph capture (the default is used
 * there without being kept); gp_batch_solve measures before it captures.
 * gp_get_radix_plan writes the plan the next length-n transform in FP32
 * (fp64 = 0: ROF, dct_poisson) or FP64 (fp64 = 1: EMD, dct_poisson_f64) will
 * use -- the default if none has been measured or set -- into radices[0..16)
 * (unused entries 0) and its pass count into *count.  gp_set_radix_plan fixes
 * a plan and exempts the length from measurement (it synchronises the
 * context stream).  GP_EUNSUPPORTED if n is not such a side in [64, 4096];
 * GP_EINVAL for NULL pointers or an invalid plan. */
int gp_get_radix_plan(gp_ctx* ctx, int fp64, int n, int* radices, int* count);
int gp_set_radix_plan(gp_ctx* ctx, int fp64, int n, const int* radices, int count);

/* ---------------------------------------------------------------- learned warm start
 * Not part of the paper.  A U-Net predicts the dual potential phi0 of the EMD
 * problem from (rho0, rho1); the iteration of section 3.2 then starts from
 * p0 = proj(grad phi0), u0 = 0 and its duality gap still decides convergence.
 *
 * Network (widths 32/64/128/256): per encoder level two 3x3 convolutions with
 * zero padding, each followed by ReLU, then 2x2 average pooling; bottleneck
 * two 3x3 conv + ReLU; per decoder level a 2x2 stride-2 transposed
 * convolution (no activation), concatenation [upsampled, encoder skip] and
 * two 3x3 conv + ReLU; a 1x1 head gives phi.  Input channels (rho0 - 1,
 * rho1 - 1).  BF16 weights and activations, FP32 accumulation (MFMA), FP32
 * master weights and Adam moments.
 *
 * Parameter blob (FP32, ws_param_count() values): layers enc0a enc0b enc1a
 * enc1b enc2a enc2b mid_a mid_b up2 dec2a dec2b up1 dec1a dec1b up0 dec0a dec0b
 * head, each weights then bias.  3x3 conv weights [cout][3][3][cin] (tap
 * (ky, kx) reads the input at offset (ky - 1, kx - 1)); transposed conv
 * weights [cin][2][2][cout] (output pixel (2y + i, 2x + j) from input (y, x)
 * through W[:, i, j, :]); head [1][32] and one bias.  (cin, cout): enc (2,32)
 * (32,32) (32,64) (64,64) (64,128) (128,128); mid (128,256) (256,256);
 * up2 (256,128); dec2 (256,128) (128,128); up1 (128,64); dec1 (128,64)
 * (64,64); up0 (64,32); dec0 (64,32) (32,32); head (32,1).
 *
 * Loss for training: mean over the batch's pixels of |grad_h phi - grad_h
 * phi*|^2 (forward differences as in the solver, h the targets' spacing). */
typedef struct ws_net ws_net;
typedef struct {
  int used_warm;      /* 1 if the reported solve started from the prediction */
  int fallback;       /* 1 if the warm start was rejected or missed max_iter and a plain solve ran */
  int warm_iters;     /* iterations of the warm attempt (0 if not tried) */
  double d0;          /* certificate value D(phi0) of the prediction */
  double seconds_predict;  /* resampling + network + certificate */
  double seconds_total;    /* whole call, including any fallback */
} ws_report;

long long ws_param_count(void);
/* Network on ctx's stream for batches of up to max_batch inputs of ny x nx
 * (multiples of 8, <= 4096; the native resolution; max_batch * ny * nx below 2^31, else
 * GP_EUNSUPPORTED).  Parameters start at 0. */
int ws_create(gp_ctx* ctx, ws_net** net, int max_batch, int ny, int nx);
int ws_destroy(ws_net* net);
/* Copy the FP32 blob (device) in (resets the Adam state) or out. */
int ws_set_params(gp_ctx* ctx, ws_net* net, const float* blob);
int ws_get_params(gp_ctx* ctx, ws_net* net, float* blob);
/* phi0 [batch][ny][nx] = net(rho0, rho1) at the native size (rho [batch][ny][nx]). */
int ws_predict(gp_ctx* ctx, ws_net* net, const float* rho0, const float* rho1, int batch, float* phi0);
/* Forward, loss against phi_star [batch][ny][nx] and parameter gradients
 * (kept for ws_adam; copied to grad, nullable, as an FP32 blob).  h > 0 is the
 * targets' grid spacing.  Synchronises; *loss receives the loss. */
int ws_grads(gp_ctx* ctx, ws_net* net, const float* rho0, const float* rho1, const float* phi_star, int batch,
             double h, float* grad, double* loss);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected) with learning
 * rate lr on the gradients of the last ws_grads. */
int ws_adam(gp_ctx* ctx, ws_net* net, double lr);
/* One training step: ws_grads (no gradient copy) then ws_adam with rate lr.
 * *loss (nullable) receives the batch's loss before the step.  Synchronises. */
int ws_train_step(gp_ctx* ctx, ws_net* net, const float* rho0, const float* rho1, const float* phi_star, int batch,
                  double h, double lr, double* loss);
/* Parameters from / to a file of ws_param_count() FP32 values, little-endian,
 * no header (the blob layout above; paper_1805_09453_amd/weights/ws_unet.f32
 * is such a file).  Loading resets the Adam state; a file that cannot be read
 * or holds another number of values gives GP_EINVAL (path and reason in
 * gp_last_error).  Both synchronise ctx's stream and use a temporary device
 * buffer of the blob's size. */
int ws_load_params(gp_ctx* ctx, ws_net* net, const char* path);
int ws_save_params(gp_ctx* ctx, ws_net* net, const char* path);
/* The resolution changes of ws_emd_solve: f x f block mean ([ny][nx] ->
 * [ny/f][nx/f], mass-preserving for densities) and bilinear interpolation
 * between cell centres ([ny][nx] -> [f ny][f nx], constant beyond the
 * outermost centres). */
int ws_downsample(gp_ctx* ctx, const float* in, int ny, int nx, int f, float* out);
int ws_upsample(gp_ctx* ctx, const float* in, int ny, int nx, int f, float* out);
/* emd_solve with the learned start.  ny, nx must be f times the network's
 * native size (f a power of two): the densities are block-averaged by f, the
 * prediction is interpolated bilinearly back (a potential in unit-square
 * units keeps its slope bound).  The start is rejected when D(phi0) <= 0;
 * a warm run that reaches opts->max_iter is followed by a plain solve with
 * the same opts (fallback).  m, phi, rep as emd_solve (phi nullable);
 * wrep nullable. */
int ws_emd_solve(gp_ctx* ctx, ws_net* net, const float* rho0, const float* rho1, float* m, float* phi, int ny,
                 int nx, double h, const gp_opts* opts, gp_report* rep, ws_report* wrep);

/* Per-kernel timing on the context's stream (a start and a stop HIP event
 * bound to each kernel's own dispatch, i.e. the kernel's execution interval;
 * for measurement, not needed by the solvers; recording is suspended inside
 * the captured graphs of gp_batch_solve).  gp_profile(ctx, 1)
 * clears and starts recording (allocates the event pool), gp_profile(ctx, 0)
 * stops.  gp_profile_read synchronises the stream and fills up to max entries
 * (one per kernel kind that ran): total elapsed ms, launch count, and the
 * algorithmic HBM bytes those launches must move (sum over launches of what
 * the kernel's definition reads and writes once).  *n_out receives the
 * number of entries.  Recording stops silently when the pool (16384 launches)
 * is full; the 'dropped' field counts unrecorded launches. */
typedef struct {
  char name[32];
  long long calls, dropped;
  double total_ms, bytes;
} gp_kstat;
int gp_profile(gp_ctx* ctx, int enable);
int gp_profile_read(gp_ctx* ctx, gp_kstat* out, int max, int* n_out);

#ifdef __cplusplus
}
#endif
#endif /* GPROX_H */
