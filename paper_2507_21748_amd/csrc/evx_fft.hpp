// Register/LDS mixed-radix FFT engine for gfx950 (wave64).
//
// A length-N complex transform is carried by TPS = N/E lanes that each hold E points.  On entry
// lane t of a sequence holds points n = t + TPS*e (e = 0..E-1) in natural order; on exit it
// holds frequencies k = t + TPS*e, also in natural order.  The transform is a Stockham autosort
// decomposition N = R_0 R_1 ... R_{S-1}: every radix divides E, so in each stage a lane runs E/R
// radix-R butterflies entirely in registers, and consecutive stages exchange data through LDS
// (S-1 exchanges; the first stage's inputs and the last stage's outputs are already where the
// lane needs them).  Twiddles between stages come from a table of exp(-2 pi i j / N) computed in
// FP64 on the host and rounded once; twiddles inside a composite radix are compile-time
// constants evaluated in FP64.
#pragma once

#include <utility>

#include "evx_device.hpp"

namespace evx {

// ------------------------------------------------------------------ compile-time helpers
template <int... Is, class F>
EVX_DEV void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
EVX_DEV void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;
// Taylor polynomials on |x| <= pi/4 (13 terms: truncation far below double rounding).
constexpr double sin_poly(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i <= 13; ++i) {
    term *= -x2 / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_poly(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i <= 13; ++i) {
    term *= -x2 / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
struct CS {
  double c, s;
};
// cos and sin of 2 pi a / b with the octant reduction done in integers.
constexpr CS cossin_frac(long a, long b) {
  a %= b;
  if (a < 0) a += b;
  const long o = (8 * a) / b;          // octant 0..7
  const long r = 8 * a - o * b;        // remainder, angle within octant = (pi/4) r / b
  const long q = o / 2;                // quadrant
  double c = 0, s = 0;
  if ((o & 1) == 0) {                  // angle within quadrant g = (pi/4) r/b in [0, pi/4)
    const double g = (kPi / 4) * double(r) / double(b);
    c = cos_poly(g);
    s = sin_poly(g);
  } else {                             // g = pi/4 + (pi/4) r/b; use pi/2 - g = (pi/4)(b-r)/b
    const double h = (kPi / 4) * double(b - r) / double(b);
    c = sin_poly(h);
    s = cos_poly(h);
  }
  switch (q) {
    case 0: return CS{c, s};
    case 1: return CS{-s, c};
    case 2: return CS{-c, -s};
    default: return CS{s, -c};
  }
}
constexpr int split_of(int R) {
  return (R % 4 == 0 && R > 4) ? 4 : (R % 2 == 0 && R > 2) ? 2 : (R % 3 == 0 && R > 3) ? 3 : 5;
}
}  // namespace ct

// v * exp(DIR * 2 pi i A / D), with exact forms for multiples of pi/2.
template <long A, long D, int DIR>
EVX_DEV float2 twmul(float2 v) {
  constexpr long a = ((A % D) + D) % D;
  if constexpr (a == 0) {
    return v;
  } else if constexpr ((4 * a) % D == 0) {
    constexpr long q = (4 * a) / D;  // 1, 2, 3 quarter turns
    if constexpr (q == 2) {
      return make_float2(-v.x, -v.y);
    } else if constexpr (q == 1) {
      return cmul_i<DIR>(v);
    } else {
      return cmul_i<-DIR>(v);
    }
  } else {
    constexpr ct::CS cs = ct::cossin_frac(a, D);
    constexpr float c = float(cs.c);
    constexpr float s = float(DIR * cs.s);
    return make_float2(__builtin_fmaf(v.x, c, -(v.y * s)), __builtin_fmaf(v.x, s, v.y * c));
  }
}

// ------------------------------------------------------------------ register DFTs
// In place, natural order in and out: X[k] = sum_n x[n] exp(DIR 2 pi i n k / R).
template <int R, int DIR>
struct Dft {
  static constexpr int R1 = ct::split_of(R);
  static constexpr int R2 = R / R1;
  static_assert(R1 * R2 == R, "radix must be 2/3/5-smooth");
  EVX_DEV static void run(float2 (&x)[R]) {
    float2 t[R];
    static_for<R2>([&](auto N2) {
      constexpr int n2 = decltype(N2)::value;
      float2 a[R1];
      static_for<R1>([&](auto N1) { a[N1] = x[R2 * N1 + n2]; });
      Dft<R1, DIR>::run(a);
      static_for<R1>([&](auto K1) {
        constexpr int k1 = decltype(K1)::value;
        t[n2 * R1 + k1] = twmul<n2 * k1, R, DIR>(a[k1]);
      });
    });
    static_for<R1>([&](auto K1) {
      constexpr int k1 = decltype(K1)::value;
      float2 b[R2];
      static_for<R2>([&](auto N2) { b[N2] = t[N2 * R1 + k1]; });
      Dft<R2, DIR>::run(b);
      static_for<R2>([&](auto K2) { x[k1 + R1 * K2] = b[K2]; });
    });
  }
};

template <int DIR>
struct Dft<1, DIR> {
  EVX_DEV static void run(float2 (&)[1]) {}
};

template <int DIR>
struct Dft<2, DIR> {
  EVX_DEV static void run(float2 (&x)[2]) {
    const float2 a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  }
};

template <int DIR>
struct Dft<3, DIR> {
  EVX_DEV static void run(float2 (&x)[3]) {
    constexpr float h = 0.866025403784438646763723170752936183f;  // sin(pi/3)
    const float2 s = cadd(x[1], x[2]);
    const float2 d = csub(x[1], x[2]);
    const float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
    const float2 r = cmul_i<DIR>(make_float2(h * d.x, h * d.y));
    x[0] = cadd(x[0], s);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  EVX_DEV static void run(float2 (&x)[4]) {
    const float2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    const float2 s13 = cadd(x[1], x[3]), d13 = cmul_i<DIR>(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  }
};

template <int DIR>
struct Dft<5, DIR> {
  EVX_DEV static void run(float2 (&x)[5]) {
    constexpr float c1 = 0.309016994374947424102293417182819059f;   // cos(2 pi / 5)
    constexpr float c2 = -0.809016994374947424102293417182819059f;  // cos(4 pi / 5)
    constexpr float s1 = 0.951056516295153572116439333379382143f;   // sin(2 pi / 5)
    constexpr float s2 = 0.587785252292473129168705954639072769f;   // sin(4 pi / 5)
    const float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    const float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    const float2 x0 = x[0];
    const float2 r1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const float2 r2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    const float2 i1 = cmul_i<DIR>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const float2 i2 = cmul_i<DIR>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    x[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
    x[1] = cadd(r1, i1);
    x[4] = csub(r1, i1);
    x[2] = cadd(r2, i2);
    x[3] = csub(r2, i2);
  }
};

// ------------------------------------------------------------------ per-length plans
// E points per lane; radices R[0..S-1] with prod R = N and every R[s] dividing E.
template <int N>
struct FftPlan;

#define EVX_FFT_PLAN(N_, E_, ...)                        \
  template <>                                            \
  struct FftPlan<N_> {                                   \
    static constexpr int E = E_;                         \
    static constexpr int TPS = N_ / E_;                  \
    static constexpr int R[] = {__VA_ARGS__};            \
    static constexpr int S = sizeof(R) / sizeof(int);    \
  };

EVX_FFT_PLAN(4, 4, 4)
EVX_FFT_PLAN(6, 6, 6)
EVX_FFT_PLAN(8, 8, 8)
EVX_FFT_PLAN(10, 10, 10)
EVX_FFT_PLAN(12, 12, 12)
EVX_FFT_PLAN(16, 16, 16)
EVX_FFT_PLAN(20, 20, 20)
EVX_FFT_PLAN(24, 12, 12, 2)
// 32, 64 and 128 take fewer points per lane than the register budget allows: they serve the
// small grids (32^3 to 128^3), where a pass has only a few waves per compute unit and more lanes
// per sequence hide more latency (128^3 step: 36.8 -> 33.5 us; 64^3: 24.3 -> 16.6 us).
EVX_FFT_PLAN(32, 8, 8, 4)
EVX_FFT_PLAN(40, 20, 20, 2)
EVX_FFT_PLAN(48, 12, 12, 4)
EVX_FFT_PLAN(50, 10, 10, 5)
EVX_FFT_PLAN(64, 4, 4, 4, 4)
EVX_FFT_PLAN(80, 20, 20, 4)
EVX_FFT_PLAN(96, 12, 12, 4, 2)
EVX_FFT_PLAN(100, 20, 20, 5)
EVX_FFT_PLAN(128, 8, 8, 8, 2)
EVX_FFT_PLAN(160, 20, 20, 4, 2)
EVX_FFT_PLAN(192, 12, 12, 4, 4)
EVX_FFT_PLAN(200, 20, 20, 10)
EVX_FFT_PLAN(256, 16, 16, 16)
EVX_FFT_PLAN(320, 20, 20, 4, 4)
EVX_FFT_PLAN(384, 12, 12, 4, 4, 2)
EVX_FFT_PLAN(400, 20, 20, 20)
EVX_FFT_PLAN(512, 8, 8, 8, 8)
EVX_FFT_PLAN(1024, 16, 16, 16, 4)

#undef EVX_FFT_PLAN

template <int N, class P = FftPlan<N>>
constexpr int plan_prefix(int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= P::R[i];
  return p;
}
template <int N, class P = FftPlan<N>>
constexpr bool plan_ok() {
  int prod = 1;
  for (int i = 0; i < P::S; ++i) {
    if (P::E % P::R[i] != 0) return false;
    prod *= P::R[i];
  }
  return prod == N && P::E * P::TPS == N;
}

// Sequences per workgroup for a length-N transform: up to 256 threads, at least 8 sequences
// (64-byte row segments) and LDS for the exchange area at most 64 KiB.
template <int N>
constexpr int seqs_per_block() {
  constexpr int tps = FftPlan<N>::TPS;
  int b = 8;
  // grow to at most 256 threads: for lane counts that are not powers of two (radix-5 plans) this
  // stops below 256 rather than above, which keeps the LDS per block small enough for more
  // resident waves (400^3 zero flux: 22% faster than 320-thread blocks)
  while (2 * b * tps <= 256 && b < 256) b *= 2;
  while (b > 8 && b * N * 8 > 65536) b /= 2;
  return b;
}

// LDS slot of point n of sequence b in the exchange area.
template <int B>
EVX_DEV int lidx(int n, int b) {
  return n * B + b;
}

// In-register/LDS transform of one sequence per lane group (see header comment).  lds must hold
// B*N float2.  The caller guarantees that no lane still reads lds when this is entered; on return
// every lane has finished its LDS accesses (the last access is followed by a barrier).
template <int N, int DIR, int B, class P = FftPlan<N>>
EVX_DEV void fft_regs(float2 (&x)[P::E], float2* lds, int b, int t,
                      const float2* EVX_RESTRICT tw) {
  static_assert(plan_ok<N, P>(), "inconsistent FFT plan");
  constexpr int E = P::E, TPS = P::TPS, S = P::S;
  static_for<S>([&](auto S_) {
    constexpr int s = decltype(S_)::value;
    constexpr int R = P::R[s];
    constexpr int p = plan_prefix<N, P>(s);
    constexpr int NB = E / R;
    constexpr int NR = N / R;
    if constexpr (s > 0) {
      static_for<NB>([&](auto I) {
        const int j = t + TPS * decltype(I)::value;
        static_for<R>([&](auto M) {
          x[decltype(I)::value + decltype(M)::value * NB] = lds[lidx<B>(j + decltype(M)::value * NR, b)];
        });
      });
      evx_sync();
    }
    static_for<NB>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const int j = t + TPS * i;
      float2 v[R];
      static_for<R>([&](auto M) { v[M] = x[i + decltype(M)::value * NB]; });
      int k = 0;
      if constexpr (s > 0) {
        k = j % p;
        const int step = k * (N / (p * R));
        static_for<R - 1>([&](auto M1) {
          constexpr int m = decltype(M1)::value + 1;
          float2 w = tw[m * step];
          if constexpr (DIR > 0) w.y = -w.y;
          v[m] = cmul(v[m], w);
        });
      }
      Dft<R, DIR>::run(v);
      if constexpr (s == S - 1) {
        static_for<R>([&](auto M) { x[i + decltype(M)::value * NB] = v[M]; });
      } else {
        const int base = (j - k) * R + k;
        static_for<R>([&](auto M) { lds[lidx<B>(base + decltype(M)::value * p, b)] = v[M]; });
      }
    });
    if constexpr (s < S - 1) evx_sync();
  });
}

}  // namespace evx
