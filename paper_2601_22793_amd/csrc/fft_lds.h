// Mixed-radix Stockham FFT over several sequences held in LDS (gfx950, 64-wide waves).
//
// COUNT sequences of length N are interleaved in LDS as buf[lds_index(j, c)] (sequence c,
// element j), so that consecutive lanes touch consecutive 8-byte words.  A stage of radix R
// with p = product of the radices already applied maps butterfly i (0 <= i < N/R) of
// sequence c as
//     inputs   x[i + q N/R],                    q = 0..R-1
//     twiddle  x_q *= W_N^(q k N/(p R)),        k = i mod p
//     outputs  y[(i - k) R + k + q p]  after an R-point DFT,
// which leaves the transform in natural order after the last stage (self-sorting).  Each
// stage is done in place: every thread first loads all its butterflies into registers, the
// workgroup synchronises, then every thread writes its outputs.  The register budget per
// thread is fixed at compile time by EMAX (upper bound of COUNT * N) and the thread count.
// Twiddles come from a table in LDS that holds W_N^j for j < N/2 (N even; all j for odd N)
// and W^(j + N/2) = -W^j for the rest, so the stages issue no global loads.
// Only forward transforms are provided; inverses use conj(FFT(conj(x))).
#pragma once

#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "epr_internal.h"

namespace epr {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i and +i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// LDS position of element j of sequence c: sequences interleaved, j * COUNT + c, with one
// unused row of COUNT values after every 32 elements (lds_rows).  The padding spreads the
// stride-R writes of a first stage (p = 1) over the LDS banks; without it all lanes of a
// wave write into the same two banks.
template <int COUNT>
__device__ __forceinline__ int lds_index(int j, int c) {
  return (j + (j >> kLdsPadShift)) * COUNT + c;
}

// lds_index(j + d, c) - lds_index(j, c) when it does not depend on j: for d a multiple of the
// padding period, and for the output offsets of a stage whose length, radix and p are powers
// of two (see fft_stage).  A compile-time constant, so such accesses take immediate offsets.
template <int COUNT>
__host__ __device__ constexpr int lds_step(int d) {
  return (d + (d >> kLdsPadShift)) * COUNT;
}
constexpr bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// All transform data and tables live in the kernel's dynamic LDS and are addressed by element
// offsets into it, never by pointers: an LDS pointer handed to an out-of-line function can lose
// its address space and turn every access into a flat access (which also waits on the vector
// memory counter, i.e. on outstanding global loads).
__device__ __forceinline__ float2* lds_f2() {
  extern __shared__ float2 lds_dyn_f2[];
  return lds_dyn_f2;
}

// Twiddles W_N^j (0 <= j < N) from the LDS table at element offset off: t[j] = W_N^j for
// j < half = tw_half(N).
struct TwTable {
  int off;
  int half;
  __device__ __forceinline__ float2 operator()(int j) const {
    const bool up = j >= half;
    const float2 w = lds_f2()[off + (up ? j - half : j)];
    return up ? make_float2(-w.x, -w.y) : w;
  }
};

// Fill the LDS table of a plan at element offset off: t[j] = tw[j * tw_stride],
// j < tw_half(n).  The caller synchronises before the first use.
__device__ __forceinline__ TwTable load_twiddles(int off, const FftPlan& plan, int tid, int nt) {
  const int half = tw_half(plan.n);
  gptr<const float2> src = G(plan.tw);
  float2* t = lds_f2() + off;
  for (int j = tid; j < half; j += nt) t[j] = ldg(src, (unsigned)(j * plan.tw_stride));
  TwTable tt;
  tt.off = off;
  tt.half = half;
  return tt;
}

// Forward R-point DFTs in registers (natural order in and out).
template <int R>
struct Dft;

template <>
struct Dft<2> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 t = u[0];
    u[0] = cadd(t, u[1]);
    u[1] = csub(t, u[1]);
  }
};

template <>
struct Dft<3> {
  __device__ __forceinline__ static void run(float2* u) {
    const float s3 = 0.86602540378443864676f;  // sin(2 pi / 3)
    float2 t1 = cadd(u[1], u[2]);
    float2 m = make_float2(u[0].x - 0.5f * t1.x, u[0].y - 0.5f * t1.y);
    float2 d = make_float2(s3 * (u[1].x - u[2].x), s3 * (u[1].y - u[2].y));
    u[0] = cadd(u[0], t1);
    u[1] = make_float2(m.x + d.y, m.y - d.x);  // m - i d
    u[2] = make_float2(m.x - d.y, m.y + d.x);  // m + i d
  }
};

template <>
struct Dft<4> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 a = cadd(u[0], u[2]), b = csub(u[0], u[2]);
    float2 c = cadd(u[1], u[3]), d = csub(u[1], u[3]);
    u[0] = cadd(a, c);
    u[2] = csub(a, c);
    u[1] = cadd(b, mul_mi(d));
    u[3] = cadd(b, mul_pi(d));
  }
};

template <>
struct Dft<5> {
  __device__ __forceinline__ static void run(float2* u) {
    const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    float2 a1 = cadd(u[1], u[4]), b1 = csub(u[1], u[4]);
    float2 a2 = cadd(u[2], u[3]), b2 = csub(u[2], u[3]);
    float2 r1 = make_float2(u[0].x + c1 * a1.x + c2 * a2.x, u[0].y + c1 * a1.y + c2 * a2.y);
    float2 r2 = make_float2(u[0].x + c2 * a1.x + c1 * a2.x, u[0].y + c2 * a1.y + c1 * a2.y);
    float2 i1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
    float2 i2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
    u[0] = make_float2(u[0].x + a1.x + a2.x, u[0].y + a1.y + a2.y);
    u[1] = cadd(r1, mul_mi(i1));
    u[4] = cadd(r1, mul_pi(i1));
    u[2] = cadd(r2, mul_mi(i2));
    u[3] = cadd(r2, mul_pi(i2));
  }
};

template <>
struct Dft<8> {
  __device__ __forceinline__ static void run(float2* u) {
    const float r = 0.70710678118654752440f;
    float2 e[4] = {u[0], u[2], u[4], u[6]};
    float2 o[4] = {u[1], u[3], u[5], u[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    // W8^1 = r (1 - i), W8^2 = -i, W8^3 = r (-1 - i)
    float2 t1 = make_float2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
    float2 t2 = mul_mi(o[2]);
    float2 t3 = make_float2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
    u[0] = cadd(e[0], o[0]);
    u[4] = csub(e[0], o[0]);
    u[1] = cadd(e[1], t1);
    u[5] = csub(e[1], t1);
    u[2] = cadd(e[2], t2);
    u[6] = csub(e[2], t2);
    u[3] = cadd(e[3], t3);
    u[7] = csub(e[3], t3);
  }
};

template <>
struct Dft<9> {
  // 9 = 3 x 3: DFT3 over n1 of u[3 n1 + n2], twiddle W9^(n2 k1), DFT3 over n2; X[k1 + 3 k2].
  __device__ __forceinline__ static void run(float2* u) {
    float2 a[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = u[3 * n1 + n2];
      Dft<3>::run(a[n2]);
    }
    // W9^1, W9^2, W9^4 (W9^j = exp(-2 pi i j / 9))
    const float2 w1 = make_float2(0.766044443118978f, -0.6427876096865393f);
    const float2 w2 = make_float2(0.17364817766693041f, -0.984807753012208f);
    const float2 w4 = make_float2(-0.9396926207859083f, -0.3420201433256689f);
    a[1][1] = cmul(a[1][1], w1);
    a[1][2] = cmul(a[1][2], w2);
    a[2][1] = cmul(a[2][1], w2);
    a[2][2] = cmul(a[2][2], w4);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      float2 b[3] = {a[0][k1], a[1][k1], a[2][k1]};
      Dft<3>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) u[k1 + 3 * k2] = b[k2];
    }
  }
};

template <>
struct Dft<15> {
  // 15 = 3 x 5 with coprime factors (Good-Thomas prime-factor mapping, no inner twiddles):
  // input n = (5 n1 + 3 n2) mod 15, output k = (10 k1 + 6 k2) mod 15, so that
  // W15^(n k) = W3^(n1 k1) W5^(n2 k2): DFT5 over n2, then DFT3 over n1.
  __device__ __forceinline__ static void run(float2* u) {
    float2 a[3][5];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < 5; ++n2) a[n1][n2] = u[(5 * n1 + 3 * n2) % 15];
      Dft<5>::run(a[n1]);
    }
#pragma unroll
    for (int k2 = 0; k2 < 5; ++k2) {
      float2 b[3] = {a[0][k2], a[1][k2], a[2][k2]};
      Dft<3>::run(b);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) u[(10 * k1 + 6 * k2) % 15] = b[k1];
    }
  }
};

template <>
struct Dft<16> {
  // 16 = 4 x 4: DFT4 over n1 of u[4 n1 + n2], twiddle W16^(n2 k1), DFT4 over n2.
  __device__ __forceinline__ static void run(float2* u) {
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = u[4 * n1 + n2];
      Dft<4>::run(a[n2]);
    }
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float r = 0.70710678118654752440f;
    // W16^1, W16^2, W16^3, W16^4(= -i), W16^6, W16^9
    const float2 w1 = make_float2(c1, -s1), w2 = make_float2(r, -r), w3 = make_float2(s1, -c1);
    const float2 w6 = make_float2(-r, -r), w9 = make_float2(-c1, s1);
    a[1][1] = cmul(a[1][1], w1);
    a[1][2] = cmul(a[1][2], w2);
    a[1][3] = cmul(a[1][3], w3);
    a[2][1] = cmul(a[2][1], w2);
    a[2][2] = mul_mi(a[2][2]);
    a[2][3] = cmul(a[2][3], w6);
    a[3][1] = cmul(a[3][1], w3);
    a[3][2] = cmul(a[3][2], w6);
    a[3][3] = cmul(a[3][3], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) u[k1 + 4 * k2] = b[k2];
    }
  }
};

// Multiply u[r] by W_N^(r t), r = 1..R-1 (r t < N).  Radix <= 5: powers of W^t by repeated
// products.  Radix 9 and 15: see below.  Radix 8 and 16: two table reads, W^t and W^(4t), and W^(4a+b) = W^(4a) W^b with
// W^2, W^3, W^8, W^12 formed by products, so each factor carries at most two roundings beyond
// the table's.  (Relative error of a 2048-point transform in FP32: about 1.1e-7, against
// 7.5e-8 with one table read per factor.)
template <int R>
__device__ __forceinline__ void apply_twiddles(float2 (&u)[R], const TwTable& tw, int t) {
  const float2 w1 = tw(t);
  if constexpr (R <= 5) {
    float2 w = w1;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      u[r] = cmul(u[r], w);
      if (r + 1 < R) w = cmul(w, w1);
    }
  } else if constexpr (R == 9 || R == 15) {
    // R = A B with B = 3 or 5: W^(B a + b) = W^(B a) W^b, powers of W^t and W^(B t) (two table
    // reads) by at most three products
    constexpr int B = R == 9 ? 3 : 5, A = R / B;
    float2 wb[B];
    wb[1] = w1;
#pragma unroll
    for (int b = 2; b < B; ++b) wb[b] = cmul(wb[b - 1], w1);
#pragma unroll
    for (int b = 1; b < B; ++b) u[b] = cmul(u[b], wb[b]);
    const float2 wB = tw(B * t);
    float2 wa = wB;
#pragma unroll
    for (int a = 1; a < A; ++a) {
      if (a == 2) wa = cmul(wB, wB);
      u[B * a] = cmul(u[B * a], wa);
#pragma unroll
      for (int b = 1; b < B; ++b) u[B * a + b] = cmul(u[B * a + b], cmul(wa, wb[b]));
    }
  } else {
    const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
    const float2 w4 = tw(4 * t);
    u[1] = cmul(u[1], w1);
    u[2] = cmul(u[2], w2);
    u[3] = cmul(u[3], w3);
    float2 wa = w4;  // W^(4a)
#pragma unroll
    for (int a = 1; a < R / 4; ++a) {
      if (a == 2) wa = cmul(w4, w4);
      if (a == 3) wa = cmul(wa, w4);
      u[4 * a] = cmul(u[4 * a], wa);
      u[4 * a + 1] = cmul(u[4 * a + 1], cmul(wa, w1));
      u[4 * a + 2] = cmul(u[4 * a + 2], cmul(wa, w2));
      u[4 * a + 3] = cmul(u[4 * a + 3], cmul(wa, w3));
    }
  }
}

// One in-place stage of radix R on COUNT interleaved sequences of length N.  p = product of
// the radices already applied, inv_p = 1/p (the butterfly's position inside its group, i mod p,
// is taken with a float reciprocal and a one-step correction: exact for i < 2^22).  FIRST: the
// stage with p = 1 (no twiddles), instantiated apart so that its register allocation does not
// carry the twiddle path.
//
// NC, PC: the length and p as compile-time constants (0: given at run time), for the lengths
// with a fixed radix sequence (fft_fixed below); all index arithmetic then folds to shifts,
// masks and immediate offsets.
template <int R, int COUNT, int NT, int EMAX, bool FIRST, int NC = 0, int PC = 0, bool STORE = false>
__device__ __forceinline__ void fft_stage(int boff, int n_rt, int p_rt, float inv_p, TwTable tw,
                                          gptr<float2> out = nullptr) {
  float2* buf = lds_f2() + boff;
  const int N = NC ? NC : n_rt;
  const int p = PC ? PC : p_rt;
  constexpr int BPT = (EMAX / R + NT - 1) / NT;
  const int T = N / R;
  const int total = COUNT * T;
  float2 u[BPT][R];
  int obase[BPT];  // first output element; its sequence is b mod COUNT
  // Compile-time length: when N / R is a multiple of the padding period, the inputs
  // i + r N/R sit at fixed distances from input 0.  When N, R and p are powers of two, so do
  // the outputs obase + r p: with a = obase, floor((a + r p) / 32) = floor(a / 32) +
  // floor(r p / 32) (for p >= 32, r p is a multiple of 32; for p < 32, a mod 32 + r p stays
  // below the next multiple of 32 because a = (i - k) R + k with 0 <= k < p and (i - k) a
  // multiple of p).
  constexpr bool kInStep = NC > 0 && (NC / R) % (1 << kLdsPadShift) == 0;
  constexpr bool kOutStep = NC > 0 && PC > 0 && is_pow2(NC) && is_pow2(R) && is_pow2(PC);
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < total) {
      const int i = b / COUNT;
      const int c = b - i * COUNT;
      if constexpr (kInStep) {
        const int ib = lds_index<COUNT>(i, c);
#pragma unroll
        for (int r = 0; r < R; ++r) u[k][r] = buf[ib + lds_step<COUNT>(r * (NC / R))];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) u[k][r] = buf[lds_index<COUNT>(i + r * T, c)];
      }
      if constexpr (FIRST) {
        obase[k] = i * R;
      } else {
        int kk;
        if constexpr (PC > 0) {
          kk = i % PC;
        } else {
          const int q = (int)((float)i * inv_p);
          kk = i - q * p;
          if (kk < 0) kk += p;
          if (kk >= p) kk -= p;
        }
        apply_twiddles<R>(u[k], tw, kk * (T / p));
        obase[k] = (i - kk) * R + kk;
      }
      Dft<R>::run(u[k]);
    }
  }
  if constexpr (STORE) {
    // last stage of a transform: the conjugated outputs go straight to global memory in
    // natural order (element e of sequence c at e COUNT + c), with no LDS pass
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
      const int b = threadIdx.x + k * NT;
      if (b < total) {
        const int c = b % COUNT;
#pragma unroll
        for (int r = 0; r < R; ++r)
          stg(out, (unsigned)((obase[k] + r * p) * COUNT + c), make_float2(u[k][r].x, -u[k][r].y));
      }
    }
    return;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < total) {
      const int c = b % COUNT;
      if constexpr (kOutStep) {
        const int ob = lds_index<COUNT>(obase[k], c);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[ob + lds_step<COUNT>(r * PC)] = u[k][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_index<COUNT>(obase[k] + r * p, c)] = u[k][r];
      }
    }
  }
  __syncthreads();
}

// Out-of-line stage: keeping each radix's stage in its own function lets the register
// allocator size it alone instead of the union of all radices live across the dispatch loop.
// TAG gives each kernel its own copies of the stage functions, so that the register budget the
// kernel declares (amdgpu_waves_per_eu) is the one the stages are scheduled for.
template <int R, int COUNT, int NT, int EMAX, int TAG, bool FIRST>
__device__ __attribute__((noinline)) void fft_stage_call(int boff, int N, int p, float inv_p,
                                                         TwTable tw) {
  fft_stage<R, COUNT, NT, EMAX, FIRST>(boff, N, p, inv_p, tw);
}

template <int COUNT, int NT, int EMAX, int TAG, bool FIRST>
__device__ __forceinline__ void fft_stage_radix(int boff, int N, int R, int p, TwTable tw) {
  const float inv_p = 1.0f / (float)p;
  switch (R) {
    case 16: fft_stage_call<16, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
    case 8: fft_stage_call<8, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
    case 4: fft_stage_call<4, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
    case 2: fft_stage_call<2, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
    case 5: fft_stage_call<5, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
    default: fft_stage_call<3, COUNT, NT, EMAX, TAG, FIRST>(boff, N, p, inv_p, tw); break;
  }
}

// Kernels whose compile-time stages are inlined (kStagesInline): the row pass (TAG 1) and the
// column pass (TAG 2).  Their register budgets hold every stage without spills, and a call
// costs more than its body's share: the caller spills scalar registers around it, the callee
// looks its dynamic LDS base up in a table and waits for every outstanding memory operation on
// entry.  Measured on a batch of 2048²-class problems: column pass -5 %, row pass -1 %.  The
// row inverse, whose own state is larger, would spill with them and keeps them out of line.
template <int TAG>
constexpr bool kStagesInline = TAG == 1 || TAG == 2;

// Compile-time stage (length N, p = P) as its own out-of-line function, and inline.
template <int R, int COUNT, int NT, int EMAX, int TAG, int N, int P>
__device__ __attribute__((noinline)) void fft_stage_fixed(int boff, TwTable tw) {
  fft_stage<R, COUNT, NT, EMAX, P == 1, N, P>(boff, N, P, 0.f, tw);
}
template <int R, int COUNT, int NT, int EMAX, int TAG, int N, int P>
__device__ __forceinline__ void fft_stage_fixed_inline(int boff, TwTable tw) {
  fft_stage<R, COUNT, NT, EMAX, P == 1, N, P>(boff, N, P, 0.f, tw);
}
template <int R, int COUNT, int NT, int EMAX, int TAG, int N, int P>
__device__ __forceinline__ void fft_stage_fixed_any(int boff, TwTable tw) {
  if constexpr (kStagesInline<TAG>)
    fft_stage_fixed_inline<R, COUNT, NT, EMAX, TAG, N, P>(boff, tw);
  else
    fft_stage_fixed<R, COUNT, NT, EMAX, TAG, N, P>(boff, tw);
}

// Stages of radices R0, Rs... of a length-N transform, starting after radices of product P.
template <int COUNT, int NT, int EMAX, int TAG, int N, int P, int R0, int... Rs>
__device__ __forceinline__ void fft_fixed(int boff, TwTable tw) {
  fft_stage_fixed_any<R0, COUNT, NT, EMAX, TAG, N, P>(boff, tw);
  if constexpr (sizeof...(Rs) > 0) fft_fixed<COUNT, NT, EMAX, TAG, N, P * R0, Rs...>(boff, tw);
}

// Compile-time last stage that writes the conjugated result to global memory (column pass).
template <int R, int COUNT, int NT, int EMAX, int TAG, int N, int P>
__device__ __forceinline__ void fft_stage_fixed_store(int boff, TwTable tw, gptr<float2> out) {
  fft_stage<R, COUNT, NT, EMAX, P == 1, N, P, true>(boff, N, P, 0.f, tw, out);
}

// As fft_fixed, with the last stage storing its conjugated outputs to global memory.
template <int COUNT, int NT, int EMAX, int TAG, int N, int P, int R0, int... Rs>
__device__ __forceinline__ void fft_fixed_store(int boff, TwTable tw, gptr<float2> out) {
  if constexpr (sizeof...(Rs) > 0) {
    fft_stage_fixed_any<R0, COUNT, NT, EMAX, TAG, N, P>(boff, tw);
    fft_fixed_store<COUNT, NT, EMAX, TAG, N, P * R0, Rs...>(boff, tw, out);
  } else {
    fft_stage_fixed_store<R0, COUNT, NT, EMAX, TAG, N, P>(boff, tw, out);
  }
}

// Stages [s_begin, s_end) of the plan in forward order (reversed = false) or of the reversed
// radix sequence (reversed = true); p is the product of the radices applied before s_begin.
// Returns the product after s_end.
template <int COUNT, int NT, int EMAX, int TAG>
__device__ __forceinline__ int fft_lds_stages(int boff, const FftPlan& plan, TwTable tw,
                                              int s_begin, int s_end, int p, bool reversed) {
  const int N = plan.n;
  for (int s = s_begin; s < s_end; ++s) {
    const int R = plan.radix[reversed ? plan.nst - 1 - s : s];
    if (p == 1)
      fft_stage_radix<COUNT, NT, EMAX, TAG, true>(boff, N, R, p, tw);
    else
      fft_stage_radix<COUNT, NT, EMAX, TAG, false>(boff, N, R, p, tw);
    p *= R;
  }
  return p;
}

// Forward FFT (unnormalised) of COUNT interleaved sequences with the given plan; EMAX bounds
// COUNT * plan.n.  Requires the caller to have synchronised after filling `buf`; returns
// synchronised.
// Lengths 512, 1024, 1280 and 2048 (the row transforms of 1024-, 2048-, 2560- and 4096-wide
// images) run compile-time stage sequences; other lengths follow the plan at run time.
// plan.variant picks one of the compiled radix orders of such a length (fft_row_variants).
template <int COUNT, int NT, int EMAX, int TAG>
__device__ __forceinline__ void fft_lds(int boff, const FftPlan& plan, TwTable tw) {
  if constexpr (COUNT * 1024 <= EMAX)
    if (plan.n == 1024) {
      if (plan.variant == 1) return fft_fixed<COUNT, NT, EMAX, TAG, 1024, 1, 8, 8, 16>(boff, tw);
      if (plan.variant == 2) return fft_fixed<COUNT, NT, EMAX, TAG, 1024, 1, 16, 16, 4>(boff, tw);
      return fft_fixed<COUNT, NT, EMAX, TAG, 1024, 1, 16, 8, 8>(boff, tw);
    }
  if constexpr (COUNT * 512 <= EMAX)
    if (plan.n == 512) {
      if (plan.variant == 1) return fft_fixed<COUNT, NT, EMAX, TAG, 512, 1, 8, 8, 8>(boff, tw);
      if (plan.variant == 2) return fft_fixed<COUNT, NT, EMAX, TAG, 512, 1, 4, 8, 16>(boff, tw);
      return fft_fixed<COUNT, NT, EMAX, TAG, 512, 1, 16, 8, 4>(boff, tw);
    }
  if constexpr (COUNT * 2048 <= EMAX)
    if (plan.n == 2048) {
      if (plan.variant == 1) return fft_fixed<COUNT, NT, EMAX, TAG, 2048, 1, 8, 16, 16>(boff, tw);
      return fft_fixed<COUNT, NT, EMAX, TAG, 2048, 1, 16, 16, 8>(boff, tw);
    }
  if constexpr (COUNT * 1280 <= EMAX)
    if (plan.n == 1280) {
      if (plan.variant == 1) return fft_fixed<COUNT, NT, EMAX, TAG, 1280, 1, 5, 16, 16>(boff, tw);
      if (plan.variant == 2) return fft_fixed<COUNT, NT, EMAX, TAG, 1280, 1, 16, 5, 16>(boff, tw);
      return fft_fixed<COUNT, NT, EMAX, TAG, 1280, 1, 16, 16, 5>(boff, tw);
    }
  fft_lds_stages<COUNT, NT, EMAX, TAG>(boff, plan, tw, 0, plan.nst, 1, false);
}

// Column filter of the preconditioner: spectral bin j of block column c is multiplied by
// scale / (1 + h (fx^2 + fy^2)), fy = signed frequency of j / ny, fx = (blk*COUNT + c) / nx.
// With m = min(j, ny - j) (so |fy| = m / ny) and a = 1 + h fx^2 for the column, the factor is
// scale / (a + (h / ny^2) m^2): m^2 < 2^24 is exact in float.
struct ColumnFilter {
  float h, scale, inv_ny, inv_nx;
  int ny, col0;
  // 1 + h fx^2 of block column c
  __device__ __forceinline__ float column_term(int c) const {
    const float fx = (float)(col0 + c) * inv_nx;
    return fmaf(h * fx, fx, 1.f);
  }
  __device__ __forceinline__ float operator()(int j, float a) const {
    const int m = min(j, ny - j);
    // hardware reciprocal (v_rcp_f32, about one ulp); the denominator is >= 1
    return scale * __builtin_amdgcn_rcpf(fmaf(h * inv_ny * inv_ny, (float)(m * m), a));
  }
};

// Fused middle of forward FFT -> filter -> inverse FFT (inverse = conj . FFT . conj with the
// radix sequence reversed).  The last forward stage (radix R, p = N/R) leaves butterfly i with
// outputs at natural positions i + q p; those are exactly the inputs of butterfly i of the
// first stage of the reversed sequence (radix R, p = 1, no twiddles).  So the filter and the
// conjugation are applied in registers and the first inverse stage follows without an LDS
// round trip.  Output layout is that of the inverse's first stage.  Inline (column pass only).
template <int R, int COUNT, int NT, int EMAX, int TAG, int NC = 0>
__device__ __forceinline__ void fft_fused_filter_stage(int boff, int n_rt, TwTable tw,
                                                                ColumnFilter filt) {
  float2* buf = lds_f2() + boff;
  const int N = NC ? NC : n_rt;
  constexpr int BPT = (EMAX / R + NT - 1) / NT;
  const int T = N / R;  // = p of the last forward stage
  const int total = COUNT * T;
  float2 u[BPT][R];
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < total) {
      const int i = b / COUNT;
      const int c = b - i * COUNT;
      if constexpr (NC > 0 && (NC / R) % (1 << kLdsPadShift) == 0) {
        const int ib = lds_index<COUNT>(i, c);
#pragma unroll
        for (int r = 0; r < R; ++r) u[k][r] = buf[ib + lds_step<COUNT>(r * (NC / R))];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) u[k][r] = buf[lds_index<COUNT>(i + r * T, c)];
      }
      // last forward stage: k = i mod p = i, twiddles W_N^(q i)
      apply_twiddles<R>(u[k], tw, i);
      Dft<R>::run(u[k]);
      // filter at natural positions i + q T, then conjugate for the inverse
      const float a = filt.column_term(c);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float H = filt(i + r * T, a);
        u[k][r] = make_float2(u[k][r].x * H, -u[k][r].y * H);
      }
      // first stage of the reversed sequence (radix R, p = 1): no twiddles
      Dft<R>::run(u[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = threadIdx.x + k * NT;
    if (b < total) {
      const int i = b / COUNT;
      const int c = b - i * COUNT;
      if constexpr (is_pow2(R) && R <= (1 << kLdsPadShift)) {
        // outputs i R + r lie in one padding period: fixed distances from output 0
        const int ob = lds_index<COUNT>(i * R, c);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[ob + lds_step<COUNT>(r)] = u[k][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_index<COUNT>(i * R + r, c)] = u[k][r];
      }
    }
  }
  __syncthreads();
}

// conj(IFFT-unnormalised(H . FFT(x))) of COUNT interleaved columns: forward stages 0..nst-2,
// the fused stage, then the remaining stages of the reversed sequence.  Compile-time lengths
// write the conjugated result (the inverse) from their last stage straight to `out`
// ([length][COUNT] complex) and return true; other lengths leave the unconjugated result in
// LDS, in place, and return false.
// Compile-time version for a length with radices R0 .. R(n-1): forward stages but the last,
// the fused stage, then the forward radices but the last, in reverse order.
template <int COUNT, int NT, int EMAX, int TAG, int N, int RL, int... Rf>
struct FusedFixed;
template <int COUNT, int NT, int EMAX, int TAG, int N, int RL, int R0, int R1>
struct FusedFixed<COUNT, NT, EMAX, TAG, N, RL, R0, R1> {
  __device__ __forceinline__ static void run(int boff, TwTable tw, const ColumnFilter& filt,
                                             gptr<float2> out) {
    fft_fixed<COUNT, NT, EMAX, TAG, N, 1, R0, R1>(boff, tw);
    fft_fused_filter_stage<RL, COUNT, NT, EMAX, TAG, N>(boff, N, tw, filt);
    fft_fixed_store<COUNT, NT, EMAX, TAG, N, RL, R1, R0>(boff, tw, out);
  }
};
template <int COUNT, int NT, int EMAX, int TAG, int N, int RL, int R0, int R1, int R2, int R3>
struct FusedFixed<COUNT, NT, EMAX, TAG, N, RL, R0, R1, R2, R3> {
  __device__ __forceinline__ static void run(int boff, TwTable tw, const ColumnFilter& filt,
                                             gptr<float2> out) {
    fft_fixed<COUNT, NT, EMAX, TAG, N, 1, R0, R1, R2, R3>(boff, tw);
    fft_fused_filter_stage<RL, COUNT, NT, EMAX, TAG, N>(boff, N, tw, filt);
    fft_fixed_store<COUNT, NT, EMAX, TAG, N, RL, R3, R2, R1, R0>(boff, tw, out);
  }
};

template <int COUNT, int NT, int EMAX, int TAG>
__device__ __forceinline__ bool fft_filter_ifft_lds(int boff, const FftPlan& plan, TwTable tw,
                                                    const ColumnFilter& filt, gptr<float2> out) {
  // column lengths 1024, 2048, 2160 and 4096 run compile-time stage sequences; plan.variant
  // picks one of the compiled radix orders (fft_col_variants)
  if constexpr (COUNT * 2048 <= EMAX)
    if (plan.n == 2048) {
      if (plan.variant == 1)
        FusedFixed<COUNT, NT, EMAX, TAG, 2048, 16, 8, 16>::run(boff, tw, filt, out);
      else if (plan.variant == 2)
        FusedFixed<COUNT, NT, EMAX, TAG, 2048, 16, 16, 8>::run(boff, tw, filt, out);
      else
        FusedFixed<COUNT, NT, EMAX, TAG, 2048, 8, 16, 16>::run(boff, tw, filt, out);
      return true;
    }
  if constexpr (COUNT * 1024 <= EMAX)
    if (plan.n == 1024) {
      if (plan.variant == 1)
        FusedFixed<COUNT, NT, EMAX, TAG, 1024, 16, 8, 8>::run(boff, tw, filt, out);
      else if (plan.variant == 2)
        FusedFixed<COUNT, NT, EMAX, TAG, 1024, 4, 16, 16>::run(boff, tw, filt, out);
      else
        FusedFixed<COUNT, NT, EMAX, TAG, 1024, 8, 16, 8>::run(boff, tw, filt, out);
      return true;
    }
  if constexpr (COUNT * 2160 <= EMAX)
    if (plan.n == 2160) {
      if (plan.variant == 1)
        FusedFixed<COUNT, NT, EMAX, TAG, 2160, 15, 9, 16>::run(boff, tw, filt, out);
      else if (plan.variant == 2)
        FusedFixed<COUNT, NT, EMAX, TAG, 2160, 9, 16, 15>::run(boff, tw, filt, out);
      else
        FusedFixed<COUNT, NT, EMAX, TAG, 2160, 15, 16, 9>::run(boff, tw, filt, out);
      return true;
    }
  if constexpr (COUNT * 4096 <= EMAX)
    if (plan.n == 4096) {
      FusedFixed<COUNT, NT, EMAX, TAG, 4096, 16, 16, 16>::run(boff, tw, filt, out);
      return true;
    }
  const int N = plan.n;
  const int last = plan.radix[plan.nst - 1];
  fft_lds_stages<COUNT, NT, EMAX, TAG>(boff, plan, tw, 0, plan.nst - 1, 1, false);
  switch (last) {
    case 16: fft_fused_filter_stage<16, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
    case 8: fft_fused_filter_stage<8, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
    case 4: fft_fused_filter_stage<4, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
    case 2: fft_fused_filter_stage<2, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
    case 5: fft_fused_filter_stage<5, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
    default: fft_fused_filter_stage<3, COUNT, NT, EMAX, TAG>(boff, N, tw, filt); break;
  }
  fft_lds_stages<COUNT, NT, EMAX, TAG>(boff, plan, tw, 1, plan.nst, last, true);
  return false;
}

}  // namespace epr
