// Register-resident FFT-based DCT-II / inverse DCT-II for gfx950.
//
// The Neumann Laplace inversion of the G-prox u-step (section 3.1 and 3.2
// updates; section 4 and appendix A: the inversion is done by FFT after even
// reflection, i.e. in the cosine basis) is a DCT-II -> diagonal scale ->
// inverse DCT-II along each axis.  Each 1-D DCT of length N is computed as
// one complex FFT of length N over TWO real sequences packed as (re, im),
// after Makhoul's even/odd reordering (J. Makhoul, "A fast cosine transform in
// one and two dimensions", IEEE TASSP 1980):
//     v_m = x_{2m},  v_{N-1-m} = x_{2m+1}           (m < N/2)
//     X_k = Re(exp(-i pi k / 2N) V_k),              V = FFT(v)
// and for the inverse
//     V_k = exp(+i pi k / 2N) (X_k - i X_{N-k}),   X_N = 0,   v = N * IFFT(V).
//
// FFT layout: a "group" of T = N/E threads owns one complex sequence; each
// thread holds E complex values in registers (E = 32 for N <= 128, E = 16 for
// longer sequences, which doubles the threads -- and the waves a CU can keep in
// flight -- for the same LDS, and halves the registers that FP64 values take).  Passes are Stockham (self-sorting,
// natural-order output) with radix H = E/2 (16 or 8), plus one leading smaller
// power-of-two pass when log2 N is not a multiple of log2 H.  Between passes
// the group exchanges through its own LDS region.  Butterfly-to-thread
// assignment:
//   * first forward pass: butterflies (b, N/R-1-b) on one thread, so the
//     Makhoul reordering is done by the global loads themselves (one float2
//     load gives x_{2m}, x_{2m+1} = v_m, v_{N-1-m});
//   * last forward pass (radix H): butterflies (b, N/H-b), so each thread holds both
//     Z_k and Z_{N-k} for the real/imaginary split and the DCT twiddle, and
//     the inverse's first pass (same radix, same indices) needs no exchange;
//   * last inverse pass: (b, N/R-1-b) again, so stores are float2 pairs.
#pragma once
#include <hip/hip_runtime.h>

namespace gp {

// ---------------------------------------------------------------- complex
// C is float2 (the per-iteration path) or double2 (the FP64 set-up solves).
template <class C> struct Cx;
template <> struct Cx<float2> { using R = float; };
template <> struct Cx<double2> { using R = double; };
template <class C> __device__ __forceinline__ C mk(typename Cx<C>::R x, typename Cx<C>::R y) {
  C c;
  c.x = x;
  c.y = y;
  return c;
}
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C conjc(C a) { return mk<C>(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, class C> __device__ __forceinline__ C mul_mi(C a) {
  return INV ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

// ---------------------------------------------------------------- small DFTs
template <bool INV, class C> __device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV, class C> __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// y_s = sum_r a_r W_R^{rs}, W_R = exp(-+2 pi i / R); in place on a[0..R)
template <int R, bool INV, class C> struct DFT;

template <bool INV, class C> struct DFT<2, INV, C> {
  __device__ __forceinline__ static void run(C* a) { dft2<INV>(a[0], a[1]); }
};
template <bool INV, class C> struct DFT<4, INV, C> {
  __device__ __forceinline__ static void run(C* a) { dft4<INV>(a[0], a[1], a[2], a[3]); }
};
template <bool INV, class C> struct DFT<8, INV, C> {
  __device__ __forceinline__ static void run(C* a) {
    using Re = typename Cx<C>::R;
    constexpr Re h = Re(0.70710678118654752440);
    constexpr Re sg = INV ? Re(1) : Re(-1);
    C e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    C o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    // W8^1 = (h, -+h), W8^2 = -+i, W8^3 = (-h, -+h)
    o1 = cmul(o1, mk<C>(h, sg * h));
    o2 = mul_mi<INV>(o2);
    o3 = cmul(o3, mk<C>(-h, sg * h));
    a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
  }
};
template <bool INV, class C> struct DFT<16, INV, C> {
  // n = r + 4m, k = s + 4q:  y_{s+4q} = sum_r W4^{rq} W16^{rs} [DFT4_m a_{r+4m}]_s
  __device__ __forceinline__ static void run(C* a) {
    using Re = typename Cx<C>::R;
    constexpr Re sg = INV ? Re(1) : Re(-1);
    constexpr Re c1 = Re(0.92387953251128675613), s1 = Re(0.38268343236508977173);
    constexpr Re h = Re(0.70710678118654752440);
#pragma unroll
    for (int r = 0; r < 4; ++r) dft4<INV>(a[r], a[r + 4], a[r + 8], a[r + 12]);
    // twiddles W16^{r s} on element (r, s) stored at a[r + 4 s]
    a[1 + 4 * 1] = cmul(a[1 + 4 * 1], mk<C>(c1, sg * s1));   // W^1
    a[1 + 4 * 2] = cmul(a[1 + 4 * 2], mk<C>(h, sg * h));     // W^2
    a[1 + 4 * 3] = cmul(a[1 + 4 * 3], mk<C>(s1, sg * c1));   // W^3
    a[2 + 4 * 1] = cmul(a[2 + 4 * 1], mk<C>(h, sg * h));     // W^2
    a[2 + 4 * 2] = mul_mi<INV>(a[2 + 4 * 2]);                // W^4
    a[2 + 4 * 3] = cmul(a[2 + 4 * 3], mk<C>(-h, sg * h));    // W^6
    a[3 + 4 * 1] = cmul(a[3 + 4 * 1], mk<C>(s1, sg * c1));   // W^3
    a[3 + 4 * 2] = cmul(a[3 + 4 * 2], mk<C>(-h, sg * h));    // W^6
    a[3 + 4 * 3] = cmul(a[3 + 4 * 3], mk<C>(-c1, -sg * s1)); // W^9
    C y[16];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      C b0 = a[0 + 4 * s], b1 = a[1 + 4 * s], b2 = a[2 + 4 * s], b3 = a[3 + 4 * s];
      dft4<INV>(b0, b1, b2, b3);
      y[s] = b0; y[s + 4] = b1; y[s + 8] = b2; y[s + 12] = b3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = y[i];
  }
};

// exp(-i pi s / 32), s = 0..15: the ratio of DCT twiddles 16 apart in a thread's
// slot (w_{b + s N/16} = w_b exp(-i pi s/32)); and exp(-i pi / 64)
constexpr double kCS32[16][2] = {
    {1.00000000000000000000, -0.00000000000000000000}, {0.99518472667219692873, -0.09801714032956060363},
    {0.98078528040323043058, -0.19509032201612824808}, {0.95694033573220882438, -0.29028467725446233105},
    {0.92387953251128673848, -0.38268343236508978178}, {0.88192126434835504956, -0.47139673682599764204},
    {0.83146961230254523567, -0.55557023301960217765}, {0.77301045336273699338, -0.63439328416364548779},
    {0.70710678118654757274, -0.70710678118654746172}, {0.63439328416364548779, -0.77301045336273699338},
    {0.55557023301960228867, -0.83146961230254523567}, {0.47139673682599780857, -0.88192126434835493853},
    {0.38268343236508983729, -0.92387953251128673848}, {0.29028467725446233105, -0.95694033573220893540},
    {0.19509032201612833135, -0.98078528040323043058}, {0.09801714032956077016, -0.99518472667219681771}};
constexpr double kE64[2] = {0.99879545620517239271, -0.04906767432741801425};

// exp(-i pi s / 2H) for s < H (H = 16 or 8): the ratio of DCT twiddles N/H apart
template <int H, class C> __device__ __forceinline__ C csh(int s) {
  using Re = typename Cx<C>::R;
  return mk<C>(Re(kCS32[s * (16 / H)][0]), Re(kCS32[s * (16 / H)][1]));
}
// exp(-i pi / 4H): the DCT twiddle of index N/2H
template <int H, class C> __device__ __forceinline__ C ceh() {
  using Re = typename Cx<C>::R;
  return H == 16 ? mk<C>(Re(kE64[0]), Re(kE64[1])) : mk<C>(Re(kCS32[16 / (2 * H)][0]), Re(kCS32[16 / (2 * H)][1]));
}
// DCT twiddle w_k = exp(-i pi k / 2N) for k = b + s N/H from w_b; and the
// partner w_{N-k} = -i conj(w_k)
template <int H, class C> __device__ __forceinline__ C dcw(C wb, int s) { return cmul(wb, csh<H, C>(s)); }
template <class C> __device__ __forceinline__ C dcw_partner(C w) { return mk<C>(-w.y, -w.x); }

// Stockham twiddles W^{j r}, r = 1..R-1, from W^j (w1) and, for R = 16, W^{4j}
// (w4): at most three roundings deep, applied to x[1..R-1]
template <int R, class C> __device__ __forceinline__ void apply_tw(C* x, C w1, C w4) {
  if constexpr (R == 2) {
    x[1] = cmul(x[1], w1);
  } else if constexpr (R == 4) {
    const C a2 = cmul(w1, w1), a3 = cmul(a2, w1);
    x[1] = cmul(x[1], w1);
    x[2] = cmul(x[2], a2);
    x[3] = cmul(x[3], a3);
  } else if constexpr (R == 8) {
    const C a2 = cmul(w1, w1), a3 = cmul(a2, w1), a4 = cmul(a2, a2);
    x[1] = cmul(x[1], w1);
    x[2] = cmul(x[2], a2);
    x[3] = cmul(x[3], a3);
    x[4] = cmul(x[4], a4);
    x[5] = cmul(x[5], cmul(a4, w1));
    x[6] = cmul(x[6], cmul(a4, a2));
    x[7] = cmul(x[7], cmul(a4, a3));
  } else {
    static_assert(R == 16, "radix");
    const C a2 = cmul(w1, w1), a3 = cmul(a2, w1);
    const C b2 = cmul(w4, w4), b3 = cmul(b2, w4);
    const C av[4] = {w1, w1, a2, a3}, bv[4] = {w4, w4, b2, b3};
#pragma unroll
    for (int r2 = 0; r2 < 4; ++r2)
#pragma unroll
      for (int r1 = 0; r1 < 4; ++r1) {
        const int r = r1 + 4 * r2;
        if (r == 0) continue;
        const C w = (r2 == 0) ? av[r1] : (r1 == 0 ? bv[r2] : cmul(av[r1], bv[r2]));
        x[r] = cmul(x[r], w);
      }
  }
}

// ---------------------------------------------------------------- schedule
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// complex values per thread for sequences of length N
constexpr int kE16MinN = 256;
template <int N> struct Sched {
  static_assert(N >= 64 && N <= 4096 && (N & (N - 1)) == 0, "power-of-two N in [64, 4096]");
  static constexpr int E = N >= kE16MinN ? 16 : 32;  // complex values per thread
  static constexpr int H = E / 2;                    // main radix, values per output slot
  static constexpr int LH = ilog2c(H);
  static constexpr int T = N / E;                    // threads per sequence
  static constexpr int L2 = ilog2c(N);
  static constexpr int REM = L2 % LH;
  static constexpr int NP = L2 / LH + (REM ? 1 : 0);
  static_assert(NP >= 2, "at least two passes");
  // forward radix of pass p; the inverse runs the sequence reversed
  static constexpr int rad(int p) { return (REM && p == 0) ? (1 << REM) : H; }
  static constexpr int irad(int p) { return rad(NP - 1 - p); }
  static constexpr int ls(int p) { int l = 1; for (int i = 0; i < p; ++i) l *= rad(i); return l; }
  static constexpr int ils(int p) { int l = 1; for (int i = 0; i < p; ++i) l *= irad(i); return l; }
  // twiddle tables: per pass, W_{LS R}^{j} for j < LS followed by W_{LS R}^{4 j}
  // (the other powers are generated in registers, see apply_tw)
  static constexpr int toff(int p) { int o = 0; for (int i = 0; i < p; ++i) o += 2 * ls(i); return o; }
  static constexpr int tsize() { return toff(NP); }
  static constexpr int itoff(int p) { int o = tsize(); for (int i = 0; i < p; ++i) o += 2 * ils(i); return o; }
  static constexpr int total_tw() { return itoff(NP); }
  // padded LDS index and per-sequence region size: one pad slot per 16 complex
  // values, and a region stride of 8 mod 32 complex values so that groups
  // interleaved lane-by-lane (the column pass) start on different banks
  static constexpr int LDS = ((N + N / 16 + 31) / 32) * 32 + 8;
};
// register array of one thread's values
template <int N, class C> using Vals = C[Sched<N>::E];

__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// One Stockham pass on NB = 32/R butterflies held by this thread.
//   inputs of butterfly b:  x[b + r N/R], twiddled by W_{LS R}^{(b mod LS) r}
//   outputs:                 y[(b/LS) LS R + (b mod LS) + s LS]
template <int N, int R, int LS, bool INV, bool FROM_LDS, bool TO_LDS, class C>
__device__ __forceinline__ void stockham_pass(Vals<N, C>& v, const int (&bi)[Sched<N>::E / R], C* lds,
                                              const C* __restrict__ tw) {
  constexpr int NB = Sched<N>::E / R;
  // twiddle bases are loaded before the LDS exchange so their latency overlaps it
  C w1[NB], w4[NB];
  if constexpr (LS > 1) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = bi[q] & (LS - 1);
      w1[q] = tw[j];
      w4[q] = (R == 16) ? tw[LS + j] : w1[q];
    }
  }
  if constexpr (FROM_LDS) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) v[q * R + r] = lds[lpad(bi[q] + r * (N / R))];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if constexpr (LS > 1) apply_tw<R>(&v[q * R], w1[q], w4[q]);
    DFT<R, INV, C>::run(&v[q * R]);
  }
  if constexpr (TO_LDS) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = bi[q] & (LS - 1);
      const int base = (bi[q] / LS) * LS * R + j;
#pragma unroll
      for (int s = 0; s < R; ++s) lds[lpad(base + s * LS)] = v[q * R + s];
    }
    __syncthreads();
  }
}

// butterfly index lists
template <int N, int R> __device__ __forceinline__ void bidx_seq(int t, int (&bi)[Sched<N>::E / R]) {
  constexpr int T = Sched<N>::T;
#pragma unroll
  for (int q = 0; q < Sched<N>::E / R; ++q) bi[q] = t + q * T;
}
template <int N, int R> __device__ __forceinline__ void bidx_mk(int t, int (&bi)[Sched<N>::E / R]) {
  constexpr int T = Sched<N>::T;
#pragma unroll
  for (int q = 0; q < Sched<N>::H / R; ++q) {
    bi[2 * q] = t + q * T;
    bi[2 * q + 1] = N / R - 1 - (t + q * T);
  }
}
template <int N, int R> __device__ __forceinline__ void bidx_dc(int t, int (&bi)[Sched<N>::E / R]) {
  constexpr int T = Sched<N>::T;
#pragma unroll
  for (int q = 0; q < Sched<N>::H / R; ++q) {
    const int b = t + q * T;
    bi[2 * q] = b;
    bi[2 * q + 1] = (b == 0) ? N / (2 * R) : N / R - b;
  }
}

// Middle passes p in [P, PEND) of the forward (INV=false) or inverse FFT.
template <int N, bool INV, int P, int PEND, class C>
__device__ __forceinline__ void middle_passes(int t, Vals<N, C>& v, C* lds, const C* __restrict__ tw) {
  if constexpr (P < PEND) {
    using S = Sched<N>;
    constexpr int R = INV ? S::irad(P) : S::rad(P);
    constexpr int LS = INV ? S::ils(P) : S::ls(P);
    constexpr int OFF = INV ? S::itoff(P) : S::toff(P);
    int bi[S::E / R];
    bidx_seq<N, R>(t, bi);
    stockham_pass<N, R, LS, INV, true, true>(v, bi, lds, tw + OFF);
    middle_passes<N, INV, P + 1, PEND, C>(t, v, lds, tw);
  }
}

// Forward DCT-II of two real sequences a, b of length N.
// ld(m, A, B) must return A = (a_{2m}, a_{2m+1}), B = (b_{2m}, b_{2m+1}) for m < N/2.
// On return, spec[slot*H + s] = (A_k, B_k) with k = dc_index(slot, s), the
// unnormalised DCT-II X_k = sum_j x_j cos(pi k (2j+1) / 2N).
template <int N, class C>
__device__ __forceinline__ void dct_split_fwd(int t, Vals<N, C>& v, C wt);

template <int N, class C, class Loader>
__device__ __forceinline__ void dct2_fwd(int t, Vals<N, C>& v, C* lds, const C* __restrict__ tw,
                                         const C* __restrict__ dctw, Loader&& ld) {
  using S = Sched<N>;
  constexpr int T = S::T, H = S::H, E = S::E;
  constexpr int R0 = S::rad(0);
  const C wt = dctw[t];  // exp(-i pi t / 2N), base of this thread's DCT twiddles
  // ---- pass 0 with the Makhoul reordering done by the loads
  {
    int bi[E / R0];
    bidx_mk<N, R0>(t, bi);
#pragma unroll
    for (int q = 0; q < H / R0; ++q) {
      const int b = t + q * T;
      const int bp = N / R0 - 1 - b;
#pragma unroll
      for (int r = 0; r < R0 / 2; ++r) {
        // m = b + r N/R0 gives input r of b and input R0-1-r of bp; m = bp + r N/R0 the converse
        C A, B;
        ld(b + r * (N / R0), A, B);
        v[(2 * q) * R0 + r] = mk<C>(A.x, B.x);
        v[(2 * q + 1) * R0 + (R0 - 1 - r)] = mk<C>(A.y, B.y);
        ld(bp + r * (N / R0), A, B);
        v[(2 * q + 1) * R0 + r] = mk<C>(A.x, B.x);
        v[(2 * q) * R0 + (R0 - 1 - r)] = mk<C>(A.y, B.y);
      }
    }
    stockham_pass<N, R0, 1, false, false, true>(v, bi, lds, tw + S::toff(0));
  }
  // ---- middle passes
  middle_passes<N, false, 1, S::NP - 1, C>(t, v, lds, tw);
  // ---- last pass (radix H), pairs (b, N/H - b): outputs stay in registers
  {
    constexpr int PL = S::NP - 1;
    int bi[2];
    bidx_dc<N, H>(t, bi);
    stockham_pass<N, H, S::ls(PL), false, true, false>(v, bi, lds, tw + S::toff(PL));
  }
  dct_split_fwd<N>(t, v, wt);
}

// Split the two real transforms held in a forward FFT's last-pass registers and
// apply exp(-i pi k / 2N).  Output s of butterfly b is index b + s N/H; Z_{N-k}
// sits at (slot1, H - 1 - s).
template <int N, class C>
__device__ __forceinline__ void dct_split_fwd(int t, Vals<N, C>& v, C wt) {
  using Re = typename Cx<C>::R;
  constexpr int H = Sched<N>::H;
  if (t != 0) {
#pragma unroll
    for (int s = 0; s < H; ++s) {
      // k0 = t + s N/H and its partner k1 = N - k0 = (N/H - t) + (H - 1 - s) N/H
      C z0 = v[s], z1 = v[H + H - 1 - s];
      C w0 = dcw<H>(wt, s), w1 = dcw_partner(w0);
      C a0 = cmul(w0, z0), c0 = cmul(w0, conjc(z1));
      C a1 = cmul(w1, z1), c1 = cmul(w1, conjc(z0));
      v[s] = mk<C>(Re(0.5) * (a0.x + c0.x), Re(0.5) * (a0.y - c0.y));
      v[H + H - 1 - s] = mk<C>(Re(0.5) * (a1.x + c1.x), Re(0.5) * (a1.y - c1.y));
    }
  } else {
    // thread 0: slot 0 holds k = s N/H (pairs s <-> H - s, s = 0 and H/2 self),
    //           slot 1 holds k = N/2H + s N/H (pairs s <-> H - 1 - s)
    C o[2 * H];
#pragma unroll
    for (int s = 0; s < H; ++s) {
      C z0 = v[s], zp = v[(H - s) & (H - 1)];
      C w0 = csh<H, C>(s);
      C a0 = cmul(w0, z0), c0 = cmul(w0, conjc(zp));
      o[s] = mk<C>(Re(0.5) * (a0.x + c0.x), Re(0.5) * (a0.y - c0.y));
      C z1 = v[H + s], zq = v[H + H - 1 - s];
      C w1 = dcw<H>(ceh<H, C>(), s);
      C a1 = cmul(w1, z1), c1 = cmul(w1, conjc(zq));
      o[H + s] = mk<C>(Re(0.5) * (a1.x + c1.x), Re(0.5) * (a1.y - c1.y));
    }
#pragma unroll
    for (int i = 0; i < 2 * H; ++i) v[i] = o[i];
  }
}

// DCT index held in spec slot (slot in {0,1}, s in [0,H)) by thread t.
template <int N> __device__ __forceinline__ int dc_index(int t, int slot, int s) {
  constexpr int H = Sched<N>::H;
  const int b = (slot == 0) ? t : ((t == 0) ? N / (2 * H) : N / H - t);
  return b + s * (N / H);
}

// Inverse of the unnormalised DCT-II, times N, for two real spectra held as
// spec[slot*H+s] = (A_k, B_k) (layout of dct2_fwd).  st(m, A, B) receives
// A = N (a_{2m}, a_{2m+1}), B = N (b_{2m}, b_{2m+1}).
template <int N, class C, class Hook>
__device__ __forceinline__ void dct2_inv_core(int t, Vals<N, C>& v, C* lds, const C* __restrict__ tw, const C wt,
                                              Hook&& before_last) {
  // wt = exp(-i pi t / 2N) (the DCT twiddle table's entry t); the inverse uses conjugates
  using Re = typename Cx<C>::R;
  using S = Sched<N>;
  constexpr int H = S::H, E = S::E;
  // ---- V_k = conj(w_k) (X_k - i X_{N-k}) for both spectra, Z_k = V^a_k + i V^b_k
  if (t != 0) {
    // pairs (slot0, s) <-> (slot1, H - 1 - s), s in [0, H)
#pragma unroll
    for (int s = 0; s < H; ++s) {
      C y0 = v[s], y1 = v[H + H - 1 - s];
      C c0 = dcw<H>(wt, s), c1 = dcw_partner(c0);
      c0.y = -c0.y;
      c1.y = -c1.y;
      C va0 = cmul(c0, mk<C>(y0.x, -y1.x)), vb0 = cmul(c0, mk<C>(y0.y, -y1.y));
      C va1 = cmul(c1, mk<C>(y1.x, -y0.x)), vb1 = cmul(c1, mk<C>(y1.y, -y0.y));
      v[s] = mk<C>(va0.x - vb0.y, va0.y + vb0.x);
      v[H + H - 1 - s] = mk<C>(va1.x - vb1.y, va1.y + vb1.x);
    }
  } else {
    C o[E];
#pragma unroll
    for (int s = 0; s < H; ++s) {
      C y0 = v[s];
      C yp = (s == 0) ? mk<C>(Re(0), Re(0)) : v[(H - s) & (H - 1)];  // X_N = 0
      C c0 = csh<H, C>(s);
      c0.y = -c0.y;
      C va = cmul(c0, mk<C>(y0.x, -yp.x)), vb = cmul(c0, mk<C>(y0.y, -yp.y));
      o[s] = mk<C>(va.x - vb.y, va.y + vb.x);
      C y1 = v[H + s], yq = v[H + H - 1 - s];
      C c1 = dcw<H>(ceh<H, C>(), s);
      c1.y = -c1.y;
      C va1 = cmul(c1, mk<C>(y1.x, -yq.x)), vb1 = cmul(c1, mk<C>(y1.y, -yq.y));
      o[H + s] = mk<C>(va1.x - vb1.y, va1.y + vb1.x);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = o[i];
  }
  // ---- inverse pass 0 (radix H) directly on the registers: butterfly b's
  // inputs b + r N/H are exactly what this thread holds
  {
    int bi[2];
    bidx_dc<N, H>(t, bi);
    stockham_pass<N, H, 1, true, false, true>(v, bi, lds, tw + S::itoff(0));
  }
  middle_passes<N, true, 1, S::NP - 1, C>(t, v, lds, tw);
  before_last();
  // ---- last inverse pass with Makhoul pairs, outputs in registers
  {
    constexpr int PL = S::NP - 1;
    constexpr int RL = S::irad(PL);
    int bi[E / RL];
    bidx_mk<N, RL>(t, bi);
    stockham_pass<N, RL, S::ils(PL), true, true, false>(v, bi, lds, tw + S::itoff(PL));
  }
}

// Positions held after dct2_inv_core: for q < H/RL and s < RL/2 the thread holds
// output pairs (x_{2m}, x_{2m+1}) for m = InvOut::m(t, q, half, s):
//   half 0: x_{2m} = v[2q RL + s],     x_{2m+1} = v[(2q+1) RL + RL-1-s],  m = b + s N/RL
//   half 1: x_{2m} = v[(2q+1) RL + s], x_{2m+1} = v[2q RL + RL-1-s],      m = bp + s N/RL
template <int N> struct InvOut {
  static constexpr int RL = Sched<N>::irad(Sched<N>::NP - 1);
  static constexpr int NQ = Sched<N>::H / RL;  // butterfly pairs per thread
  static constexpr int NS = RL / 2;            // outputs per butterfly
  __device__ __forceinline__ static int m(int t, int q, int half, int s) {
    const int b = t + q * Sched<N>::T;
    return (half ? N / RL - 1 - b : b) + s * (N / RL);
  }
  template <class C> __device__ __forceinline__ static void get(const Vals<N, C>& v, int q, int half, int s, C& x0,
                                                                 C& x1) {
    x0 = v[(2 * q + half) * RL + s];
    x1 = v[(2 * q + 1 - half) * RL + (RL - 1 - s)];
  }
};

template <int N, class C, class Storer>
__device__ __forceinline__ void dct2_inv(int t, Vals<N, C>& v, C* lds, const C* __restrict__ tw, const C wt,
                                         Storer&& st) {
  using S = Sched<N>;
  constexpr int T = S::T;
  dct2_inv_core<N>(t, v, lds, tw, wt, [] {});
  {
    constexpr int RL = S::irad(S::NP - 1);
#pragma unroll
    for (int q = 0; q < S::H / RL; ++q) {
      const int b = t + q * T;
      const int bp = N / RL - 1 - b;
#pragma unroll
      for (int s = 0; s < RL / 2; ++s) {
        C x0 = v[(2 * q) * RL + s], x1 = v[(2 * q + 1) * RL + (RL - 1 - s)];
        st(b + s * (N / RL), mk<C>(x0.x, x1.x), mk<C>(x0.y, x1.y));
        C y0 = v[(2 * q + 1) * RL + s], y1 = v[(2 * q) * RL + (RL - 1 - s)];
        st(bp + s * (N / RL), mk<C>(y0.x, y1.x), mk<C>(y0.y, y1.y));
      }
    }
  }
}

}  // namespace gp
