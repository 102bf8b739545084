// Device FFT building blocks for gfx950: compile-time mixed-radix Stockham
// passes through LDS, with each pass's radix-R DFT done in registers.
//
// A length-N transform is factored N = R0 * R1 (* R2); pass s reads R
// elements spaced N/R apart, multiplies by e^{-2 pi i k r/(Ns R)} (Ns = the
// product of the earlier radices, k = butterfly index mod Ns), runs a radix-R
// DFT in registers and writes the results Ns apart (self-sorting: natural
// order in, natural order out). Composite radices (16, 20, 21, 32, ...) are
// themselves split Cooley-Tukey style with constant twiddles, fully unrolled,
// so one LDS round trip covers several radix stages.
//
// All transforms here are forward (e^{-i}); an inverse transform is done as
// conj(FFT(conj(x))), with both conjugations folded into the surrounding
// loads and stores.
#pragma once
#include <hip/hip_runtime.h>

namespace dh {

// ------------------------------------------------------------------ constexpr trig
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin_reduced(double x) {  // |x| <= pi/4
  double term = x, sum = x;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_reduced(double x) {  // |x| <= pi/4
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 14; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi num/den for integers, exact octant reduction
constexpr double ct_cos2pi(long num, long den) {
  long n = ((num % den) + den) % den;       // [0, den)
  // reduce with symmetries on 8*n/den
  long o = (8 * n) / den;                   // octant 0..7
  double x = 2.0 * kPi * double(n) / double(den);
  switch (o) {
    case 0: return ct_cos_reduced(x);
    case 1: return ct_sin_reduced(kPi / 2 - x);
    case 2: return -ct_sin_reduced(x - kPi / 2);
    case 3: return -ct_cos_reduced(kPi - x);
    case 4: return -ct_cos_reduced(x - kPi);
    case 5: return -ct_sin_reduced(3 * kPi / 2 - x);
    case 6: return ct_sin_reduced(x - 3 * kPi / 2);
    default: return ct_cos_reduced(2 * kPi - x);
  }
}
constexpr double ct_sin2pi(long num, long den) { return ct_cos2pi(num * 4 - den, 4 * den); }

// ------------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // * (-i)

// multiply by the constant e^{-2 pi i e/R}
template <int E, int R>
__device__ __forceinline__ float2 twc(float2 a) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == R) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * e == R) {
    return mul_mi(a);
  } else if constexpr (4 * e == 3 * R) {
    return make_float2(-a.y, a.x);
  } else {
    constexpr float c = (float)ct_cos2pi(e, R);
    constexpr float s = (float)(-ct_sin2pi(e, R));
    return make_float2(fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c));
  }
}

// ------------------------------------------------------------------ base butterflies (forward)
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
__device__ __forceinline__ void dft4(float2* v) {
  float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  float2 c = cadd(v[1], v[3]), d = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  constexpr float h = 0.70710678118654752440f;
  float2 o1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = mul_mi(o[2]);
  float2 o3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}
// cos / sin of 2 pi m / R, m < R, evaluated at compile time
template <int R>
struct RootTable {
  float c[R], s[R];
  constexpr RootTable() : c(), s() {
    for (int m = 0; m < R; ++m) {
      c[m] = (float)ct_cos2pi(m, R);
      s[m] = (float)ct_sin2pi(m, R);
    }
  }
};

// odd prime radix: y_k = x0 + sum_j [(x_j + x_{R-j}) cos - i (x_j - x_{R-j}) sin]
template <int R>
__device__ __forceinline__ void dft_odd(float2* v) {
  constexpr int H = (R - 1) / 2;
  constexpr RootTable<R> K{};
  float2 s[H + 1], d[H + 1];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    s[j] = cadd(v[j], v[R - j]);
    d[j] = csub(v[j], v[R - j]);
  }
  float2 x0 = v[0];
  float2 y0 = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) y0 = cadd(y0, s[j]);
  float2 out[R];
  out[0] = y0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    float2 a = x0, b = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const float c = K.c[(j * k) % R];
      const float sn = K.s[(j * k) % R];
      a.x = fmaf(c, s[j].x, a.x);
      a.y = fmaf(c, s[j].y, a.y);
      b.x = fmaf(sn, d[j].x, b.x);
      b.y = fmaf(sn, d[j].y, b.y);
    }
    out[k] = make_float2(a.x + b.y, a.y - b.x);
    out[R - k] = make_float2(a.x - b.y, a.y + b.x);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) v[k] = out[k];
}

constexpr bool is_base_radix(int r) {
  return r == 1 || r == 2 || r == 3 || r == 4 || r == 5 || r == 7 || r == 8 || r == 11 || r == 13;
}
constexpr int split_radix(int r) {
  return (r % 8 == 0 && r != 16) ? 8 : (r % 4 == 0) ? 4 : (r % 2 == 0) ? 2 : (r % 3 == 0) ? 3 : (r % 5 == 0) ? 5 : (r % 7 == 0) ? 7 : (r % 11 == 0) ? 11 : 13;
}

template <int R, int R1, int R2, int I = 0>
__device__ __forceinline__ void static_for_tw(float2* y) {
  if constexpr (I < R1 * R2) {
    constexpr int n2 = I / R1, k1 = I % R1;
    y[I] = twc<n2 * k1, R>(y[I]);
    static_for_tw<R, R1, R2, I + 1>(y);
  }
}

// radix-R DFT of v[0..R) in registers (forward)
template <int R>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2(v);
  } else if constexpr (R == 4) {
    dft4(v);
  } else if constexpr (R == 8) {
    dft8(v);
  } else if constexpr (is_base_radix(R)) {
    dft_odd<R>(v);
  } else {
    constexpr int R1 = split_radix(R);
    constexpr int R2 = R / R1;
    float2 y[R];
    // inner length-R1 DFTs over n1 for each n2 (x index n = R2 n1 + n2)
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
      dft<R1>(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = t[k1];
    }
    // twiddles e^{-2 pi i n2 k1 / R}
    static_for_tw<R, R1, R2>(y);
    // outer length-R2 DFTs over n2 for each k1; output index k1 + R1 k2
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2 * R1 + k1];
      dft<R2>(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
}

// ------------------------------------------------------------------ Stockham pass over NTR transforms
// LDS layout of one transform (Lds<N> below). Measured bank behaviour of the
// gfx950 LDS: 64-bit reads serve 32 lanes per cycle over 32 banks of 8 bytes,
// 64-bit writes 16 lanes per cycle over 32 banks of 4 bytes (so a float2 slot
// is bank (index mod 32) for reads, (index mod 16) for writes). Two layouts:
//  - padded: element i at i + i / PAD (one spare slot after every PAD = R0
//    elements), transform t at t * STRIDE (odd STRIDE >= the padded length);
//  - swizzled (512 = 8 x 8 x 8, 1024 = 16 x 8 x 8, 2048 = 16 x 16 x 8):
//    element i at i XOR s(i), no spare slots, STRIDE = N + 4. For 512, s moves
//    bits 4..6 onto bits 0..2 and bit 6 onto bit 3; for the plans that start
//    with radix 16, s moves bits 4..7 onto bits 0..3. Every pass's reads (32
//    consecutive elements) and writes (runs of 16 lanes: R0-element blocks in
//    the first pass, groups of NS lanes in the later ones) then fall in
//    distinct banks, and the stride of 4 mod 32 spreads the transforms of a
//    workgroup over the banks for reads across transforms.
template <int PAD>
__device__ __forceinline__ int padi(int i) { return i + i / PAD; }
template <int N>
__host__ __device__ constexpr int swz(int i) {
  return N == 512 ? i ^ ((i >> 4) & 7) ^ (((i >> 6) & 1) << 3) : i ^ ((i >> 4) & 15);
}

// a twiddle-table entry from LDS / generic memory, or from the global address
// space (read as a plain vector: the float2 class cannot be copied from there)
typedef float tw_floatx2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_tw(const float2* __restrict__ t, int i) { return t[i]; }
__device__ __forceinline__ float2 ld_tw(const __attribute__((address_space(1))) float2* t, int i) {
  const tw_floatx2 v = reinterpret_cast<const __attribute__((address_space(1))) tw_floatx2*>(t)[i];
  return make_float2(v.x, v.y);
}

// buf: LDS; tw: this pass's twiddle table (see fft_lds), in LDS or, where a
// workgroup's LDS is better spent on occupancy, in global memory (TW is then a
// global-address-space pointer, read through the caches).
template <int N> struct Lds;

// ROT (last pass only, NS R = N): the outputs go out in plain order, rotated
// down by `rot` blocks of NS: bin b + NS r to slot b + NS ((r - rot) mod R).
template <int N, int R, int NS, int NTR, int STRIDE, int TPB, typename TW, bool ROT = false>
__device__ __forceinline__ void stockham_pass(float2* buf, TW tw, int tid, int rot = 0) {
  static_assert(!ROT || NS * R == N, "rotated output from the last pass only");
  constexpr int NB = N / R;
  constexpr int TOTAL = NTR * NB;
  constexpr int IT = (TOTAL + TPB - 1) / TPB;
  float2 v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * TPB;
    if (TOTAL % TPB == 0 || g < TOTAL) {
      const int tr = g / NB, b = g % NB;
      const float2* src = buf + tr * STRIDE;
      if constexpr (Lds<N>::SWZ) {
        const int fa = Lds<N>::at(b);
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = src[Lds<N>::join(fa, r * NB)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = src[Lds<N>::at(b + r * NB)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * TPB;
    if (TOTAL % TPB == 0 || g < TOTAL) {
      const int tr = g / NB, b = g % NB;
      const int k = b % NS;
      if constexpr (NS > 1) {
        // this pass's twiddles e^{-2 pi i k r/(NS R)}, stored [r-1][k]
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], ld_tw(tw, (r - 1) * NS + k));
      }
      dft<R>(v[it]);
      float2* dst = buf + tr * STRIDE;
      const int base = (b / NS) * NS * R + k;
      if constexpr (ROT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int rr = r - rot < 0 ? r - rot + R : r - rot;    // uniform across the workgroup
          dst[k + rr * NS] = v[it][r];
        }
      } else if constexpr (Lds<N>::SWZ) {
        const int fa = Lds<N>::at(base);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[Lds<N>::join(fa, r * NS)] = v[it][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) dst[Lds<N>::at(base + r * NS)] = v[it][r];
      }
    }
  }
  __syncthreads();
}

// Factorisations (radices per pass) of the supported lengths.
template <int N> struct FftPlan;
template <> struct FftPlan<16>   { static constexpr int R0 = 16, R1 = 1,  R2 = 1; };
template <> struct FftPlan<32>   { static constexpr int R0 = 8,  R1 = 4,  R2 = 1; };
template <> struct FftPlan<48>   { static constexpr int R0 = 6,  R1 = 8,  R2 = 1; };
template <> struct FftPlan<64>   { static constexpr int R0 = 8,  R1 = 8,  R2 = 1; };
template <> struct FftPlan<96>   { static constexpr int R0 = 12, R1 = 8,  R2 = 1; };
template <> struct FftPlan<112>  { static constexpr int R0 = 16, R1 = 7,  R2 = 1; };
template <> struct FftPlan<128>  { static constexpr int R0 = 16, R1 = 8,  R2 = 1; };
template <> struct FftPlan<176>  { static constexpr int R0 = 16, R1 = 11, R2 = 1; };
template <> struct FftPlan<208>  { static constexpr int R0 = 16, R1 = 13, R2 = 1; };
template <> struct FftPlan<256>  { static constexpr int R0 = 16, R1 = 16, R2 = 1; };
template <> struct FftPlan<320>  { static constexpr int R0 = 16, R1 = 20, R2 = 1; };
template <> struct FftPlan<336>  { static constexpr int R0 = 16, R1 = 21, R2 = 1; };
template <> struct FftPlan<512>  { static constexpr int R0 = 8,  R1 = 8,  R2 = 8; };
template <> struct FftPlan<640>  { static constexpr int R0 = 8,  R1 = 8,  R2 = 10; };
template <> struct FftPlan<672>  { static constexpr int R0 = 32, R1 = 21, R2 = 1; };
template <> struct FftPlan<1024> { static constexpr int R0 = 16, R1 = 8,  R2 = 8; };
template <> struct FftPlan<2048> { static constexpr int R0 = 16, R1 = 16, R2 = 8; };

// layout of a length-N transform in LDS (see stockham_pass)
template <int N> struct Lds {
  static constexpr bool SWZ = N == 512 || N == 1024 || N == 2048;
  static constexpr int PAD = FftPlan<N>::R0;
  static constexpr int SPAN = SWZ ? N : N + (N - 1) / PAD + 1;  // slots one transform covers
  static constexpr int STRIDE = SWZ ? N + 4 : SPAN | 1;         // transform stride
  __device__ static __forceinline__ int at(int i) {
    if constexpr (SWZ)
      return swz<N>(i);
    else
      return padi<PAD>(i);
  }
  // swizzled layout: at(a + c) for a lane part a and a compile-time part c
  // with no common bits, given fa = at(a). The swizzle is linear over XOR and
  // changes bits 0..3 only, so at(a + c) = fa ^ at(c); where fa has no bits
  // in at(c)'s bits 4 and up (true for every split the passes make: the
  // constant part sits above the lane part's bits, or between its groups of
  // bits with at(a) clear there), that XOR is a small XOR plus an add, which
  // folds into the LDS instruction's immediate offset.
  __device__ static __forceinline__ int join(int fa, int c) {
    const int ac = swz<N>(c);
    return (fa ^ (ac & 15)) + (ac & ~15);
  }
};

// ---------------------------------------------------------------------------
// Pass 1 with its operands already in registers. For butterfly g = tid + it*TPB
// (< NTR * N/R0): transform tr = g / (N/R0), b = g % (N/R0), and v[it][r] must
// hold element b + r * N/R0 of transform tr. Runs the radix-R0 DFT and writes
// the results to LDS (padded layout of Lds<N>); no barrier.
template <int N, int NTR, int TPB>
struct Pass1 {
  static constexpr int R0 = FftPlan<N>::R0;
  static constexpr int NB = N / R0;
  static constexpr int TOTAL = NTR * NB;
  static constexpr int IT = (TOTAL + TPB - 1) / TPB;
};

template <int N, int NTR, int STRIDE, int TPB>
__device__ __forceinline__ void fft_pass1_regs(float2 (*v)[FftPlan<N>::R0], float2* buf, int tid) {
  using Q = Pass1<N, NTR, TPB>;
  constexpr int R0 = Q::R0, NB = Q::NB;
#pragma unroll
  for (int it = 0; it < Q::IT; ++it) {
    const int g = tid + it * TPB;
    if (Q::TOTAL % TPB == 0 || g < Q::TOTAL) {
      const int tr = g / NB, b = g % NB;
      dft<R0>(v[it]);
      if constexpr (Lds<N>::SWZ) {
        // at(b R0 + r) = at(b R0) ^ r: the swizzle reads bits above the first radix
        // (in bytes, so that the XOR and the transform offset fold into one add)
        char* dst = reinterpret_cast<char*>(buf + tr * STRIDE);
        const int a8 = Lds<N>::at(b * R0) * 8;
#pragma unroll
        for (int r = 0; r < R0; ++r) *reinterpret_cast<float2*>(dst + (a8 ^ (r * 8))) = v[it][r];
      } else {
        float2* dst = buf + tr * STRIDE + padi<R0>(b * R0);
#pragma unroll
        for (int r = 0; r < R0; ++r) dst[r] = v[it][r];   // padi(b R0 + r) = padi(b R0) + r
      }
    }
  }
}

// Passes 2.. of the transform (starts and ends with a barrier).
template <int N, int NTR, int STRIDE, int TPB, typename TW>
__device__ __forceinline__ void fft_rest(float2* buf, TW tw, int tid) {
  using P = FftPlan<N>;
  __syncthreads();
  if constexpr (P::R1 > 1) stockham_pass<N, P::R1, P::R0, NTR, STRIDE, TPB>(buf, tw, tid);
  constexpr int OFF2 = (P::R1 - 1) * P::R0;
  if constexpr (P::R2 > 1) stockham_pass<N, P::R2, P::R0 * P::R1, NTR, STRIDE, TPB>(buf, tw + OFF2, tid);
}

// Passes 2.. as fft_rest, the last one writing its outputs in plain order,
// rotated so that bin (rot NSL + i) mod N lands at slot i of the transform
// (NSL = the last pass's NS = N / its radix; 0 <= rot < that radix). Needs a
// plan of two or more passes.
template <int N> constexpr int last_ns() {
  return FftPlan<N>::R2 > 1 ? FftPlan<N>::R0 * FftPlan<N>::R1 : FftPlan<N>::R0;
}
template <int N, int NTR, int STRIDE, int TPB, typename TW>
__device__ __forceinline__ void fft_rest_rot(float2* buf, TW tw, int tid, int rot) {
  using P = FftPlan<N>;
  static_assert(P::R1 > 1, "a single-pass plan has no later pass to rotate");
  __syncthreads();
  if constexpr (P::R2 > 1) {
    stockham_pass<N, P::R1, P::R0, NTR, STRIDE, TPB>(buf, tw, tid);
    constexpr int OFF2 = (P::R1 - 1) * P::R0;
    stockham_pass<N, P::R2, P::R0 * P::R1, NTR, STRIDE, TPB, TW, true>(buf, tw + OFF2, tid, rot);
  } else {
    stockham_pass<N, P::R1, P::R0, NTR, STRIDE, TPB, TW, true>(buf, tw, tid, rot);
  }
}

// forward FFT of NTR transforms of length N held in LDS (padded layout of
// Lds<N>, transform t at buf + t * STRIDE). tw holds the twiddles of pass 2
// then pass 3: entry (r-1)*NS + k = e^{-2 pi i k r / (NS R)}, so the lanes of
// a wave (consecutive k) read consecutive entries.
template <int N, int NTR, int STRIDE, int TPB, typename TW>
__device__ __forceinline__ void fft_lds(float2* buf, TW tw, int tid) {
  using P = FftPlan<N>;
  static_assert(P::R0 * P::R1 * P::R2 == N, "bad factorisation");
  static_assert(STRIDE >= Lds<N>::SPAN, "stride too small");
  stockham_pass<N, P::R0, 1, NTR, STRIDE, TPB>(buf, tw, tid);
  if constexpr (P::R1 > 1) stockham_pass<N, P::R1, P::R0, NTR, STRIDE, TPB>(buf, tw, tid);
  constexpr int OFF2 = (P::R1 - 1) * P::R0;
  if constexpr (P::R2 > 1) stockham_pass<N, P::R2, P::R0 * P::R1, NTR, STRIDE, TPB>(buf, tw + OFF2, tid);
}

}  // namespace dh
