// Register/LDS Stockham FFT building blocks for gfx950 (wave64).
//
// A "line" (one row or one column of a wave image, or one q's time series) of length N is held by
// L lanes of one wavefront, E = N / L complex values per lane, in *striped* order: lane l holds
// elements l + L*j in register j.  A plan is a list of radices R_1..R_m with product N, each
// dividing E.  Stage k (radix R, NS = R_1*...*R_{k-1}) performs the N/R radix-R butterflies of the
// Stockham autosort formulation: butterfly b reads elements b + (N/R)*r, multiplies them by the
// twiddles exp(-+2 pi i (b mod NS) r / (NS R)), applies a length-R DFT and writes its outputs to
// (b/NS)*NS*R + (b mod NS) + r*NS.  Lane l owns butterflies b = l + L*i (i < E/R); their inputs are
// all in its own registers when the data are striped, and after the last stage the outputs are
// striped again, so only the m-1 intermediate stages exchange data through LDS.  The lines of a
// wave never share LDS, so no workgroup barrier is needed inside a transform.
//
// Lengths with odd factors (560 = 4 x 5 x 4 x 7 on 28 lanes, 1000 = 4 x 5 x 5 x 10 on 50 lanes)
// use the same scheme with one extension: the last radix need not divide E.  The last stage of a Stockham plan reads and writes
// the same positions b + (N/R) r, so it can run in place in the line's LDS region, each lane taking
// butterflies b = l, l + L, ... in rounds.  All twiddles of such a plan come from a table of the
// N-th roots of unity that the workgroup keeps in LDS (exp(-2 pi i m / N) at m; a stage of span NS
// and radix R reads entry (b mod NS) r N / (NS R)).  L need not divide 64 either (the lanes past
// the last whole line of a wavefront stay idle).
//
// The per-lane pieces (butterflies, output positions, twiddle generation) are __host__ __device__
// so that a CPU emulation of the lanes can check the index algebra against a plain DFT.
#pragma once
#include <hip/hip_runtime.h>

#define TACAW_HD __host__ __device__ __forceinline__

namespace tacaw {

TACAW_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
TACAW_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
TACAW_HD float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
TACAW_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
TACAW_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
TACAW_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV> TACAW_HD float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// exp(-i pi/4) (forward) / exp(+i pi/4) (inverse) times a
template <bool INV> TACAW_HD float2 mul_w8(float2 a) {
  const float h = 0.70710678118654752440f;
  return INV ? make_float2((a.x - a.y) * h, (a.x + a.y) * h)
             : make_float2((a.x + a.y) * h, (a.y - a.x) * h);
}

// exp(-+2 pi i J / 16) times a, J a compile-time constant in [0, 16)
template <bool INV, int J> TACAW_HD float2 mul_w16(float2 a) {
  constexpr int j = J & 15;
  if constexpr (j == 0) return a;
  else if constexpr (j == 4) return mul_mi<INV>(a);
  else if constexpr (j == 8) return make_float2(-a.x, -a.y);
  else if constexpr (j == 12) return mul_mi<!INV>(a);
  else if constexpr (j == 2) return mul_w8<INV>(a);
  else if constexpr (j == 6) return mul_mi<INV>(mul_w8<INV>(a));
  else if constexpr (j == 10) return make_float2(-mul_w8<INV>(a).x, -mul_w8<INV>(a).y);
  else if constexpr (j == 14) return mul_mi<!INV>(mul_w8<INV>(a));
  else {
    // odd multiples of pi/8
    const float c1 = 0.92387953251128675613f;  // cos(pi/8)
    const float s1 = 0.38268343236508977173f;  // sin(pi/8)
    constexpr int q = j % 4;                   // 1 or 3 within the quadrant
    float c = (q == 1) ? c1 : s1;
    float s = (q == 1) ? s1 : c1;
    // w = exp(-i theta) with theta = (j mod 4) pi/8, then rotate by the quadrant
    float2 w = INV ? make_float2(c, s) : make_float2(c, -s);
    float2 r = cmul(a, w);
    constexpr int quad = j / 4;
    if constexpr (quad == 0) return r;
    else if constexpr (quad == 1) return mul_mi<INV>(r);
    else if constexpr (quad == 2) return make_float2(-r.x, -r.y);
    else return mul_mi<!INV>(r);
  }
}

// In-place length-R DFT, natural order in and out.
template <int R, bool INV> TACAW_HD void dft(float2* x);

template <> TACAW_HD void dft<2, false>(float2* x) {
  float2 a = x[0], b = x[1];
  x[0] = cadd(a, b); x[1] = csub(a, b);
}
template <> TACAW_HD void dft<2, true>(float2* x) { dft<2, false>(x); }

template <bool INV> TACAW_HD void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  float2 t2 = cadd(x1, x3), t3 = mul_mi<INV>(csub(x1, x3));
  x0 = cadd(t0, t2); x2 = csub(t0, t2);
  x1 = cadd(t1, t3); x3 = csub(t1, t3);
}
template <> TACAW_HD void dft<4, false>(float2* x) { dft4<false>(x[0], x[1], x[2], x[3]); }
template <> TACAW_HD void dft<4, true>(float2* x) { dft4<true>(x[0], x[1], x[2], x[3]); }

// 8 = 2 x 4: n = n1 + 2 n2, k = 4 k1 + k2
template <bool INV> TACAW_HD void dft8(float2* x) {
  float2 a0 = x[0], a1 = x[2], a2 = x[4], a3 = x[6];
  float2 b0 = x[1], b1 = x[3], b2 = x[5], b3 = x[7];
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  b1 = mul_w8<INV>(b1);
  b2 = mul_mi<INV>(b2);
  b3 = mul_mi<INV>(mul_w8<INV>(b3));
  x[0] = cadd(a0, b0); x[4] = csub(a0, b0);
  x[1] = cadd(a1, b1); x[5] = csub(a1, b1);
  x[2] = cadd(a2, b2); x[6] = csub(a2, b2);
  x[3] = cadd(a3, b3); x[7] = csub(a3, b3);
}
template <> TACAW_HD void dft<8, false>(float2* x) { dft8<false>(x); }
template <> TACAW_HD void dft<8, true>(float2* x) { dft8<true>(x); }

// 16 = 4 x 4: n = n1 + 4 n2, k = 4 k1 + k2
template <bool INV> TACAW_HD void dft16(float2* x) {
  float2 y[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 a = x[n1], b = x[n1 + 4], c = x[n1 + 8], d = x[n1 + 12];
    dft4<INV>(a, b, c, d);
    y[n1 * 4 + 0] = a; y[n1 * 4 + 1] = b; y[n1 * 4 + 2] = c; y[n1 * 4 + 3] = d;
  }
  // twiddles W16^(n1 k2)
  y[5] = mul_w16<INV, 1>(y[5]);   y[6] = mul_w16<INV, 2>(y[6]);   y[7] = mul_w16<INV, 3>(y[7]);
  y[9] = mul_w16<INV, 2>(y[9]);   y[10] = mul_w16<INV, 4>(y[10]); y[11] = mul_w16<INV, 6>(y[11]);
  y[13] = mul_w16<INV, 3>(y[13]); y[14] = mul_w16<INV, 6>(y[14]); y[15] = mul_w16<INV, 9>(y[15]);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 a = y[k2], b = y[4 + k2], c = y[8 + k2], d = y[12 + k2];
    dft4<INV>(a, b, c, d);
    x[k2] = a; x[4 + k2] = b; x[8 + k2] = c; x[12 + k2] = d;
  }
}
template <> TACAW_HD void dft<16, false>(float2* x) { dft16<false>(x); }
template <> TACAW_HD void dft<16, true>(float2* x) { dft16<true>(x); }

// cos and sin of 2 pi m / n in double precision at compile time: reduction to the nearest quarter
// turn with an exact integer numerator, then Taylor series on |r| <= pi/4
constexpr double ct_sincos2pi(long m, long n, bool want_sin) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m + n / 2) / n;                        // nearest quarter turn
  const double r = (double)(4 * m - q * n) * 3.14159265358979323846 / (2.0 * (double)n);
  double ts = r, tc = 1.0, es = r, ec = 1.0;
  for (int k = 1; k < 12; ++k) {
    es *= -r * r / (double)((2 * k) * (2 * k + 1));
    ec *= -r * r / (double)((2 * k - 1) * (2 * k));
    ts += es;
    tc += ec;
  }
  switch (q & 3) {
    case 0: return want_sin ? ts : tc;
    case 1: return want_sin ? tc : -ts;
    case 2: return want_sin ? -ts : -tc;
    default: return want_sin ? -tc : ts;
  }
}

// cos and sin of 2 pi j / N, j < N, as float constants
template <int N> struct RootTable {
  float c[N], s[N];
  constexpr RootTable() : c(), s() {
    for (int j = 0; j < N; ++j) {
      c[j] = (float)ct_sincos2pi(j, N, false);
      s[j] = (float)ct_sincos2pi(j, N, true);
    }
  }
};
template <int N> inline constexpr RootTable<N> kRoots{};

// exp(-+2 pi i j / N) (forward / inverse), j reduced mod N at compile time
template <int N, bool INV> TACAW_HD float2 root(int j) {
  const int k = ((j % N) + N) % N;
  return INV ? make_float2(kRoots<N>.c[k], kRoots<N>.s[k]) : make_float2(kRoots<N>.c[k], -kRoots<N>.s[k]);
}

// odd prime R: inputs paired as a_m = x_m + x_{R-m}, b_m = x_m - x_{R-m}; then
// X_k = x_0 + sum_m a_m cos(2 pi m k / R) -+ i sum_m b_m sin(2 pi m k / R) and X_{R-k} with the
// other sign (upper signs forward)
template <int R, bool INV> TACAW_HD void dft_prime(float2* x) {
  constexpr int H = (R - 1) / 2;
  float2 a[H], b[H];
  float2 sum = x[0];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    a[m - 1] = cadd(x[m], x[R - m]);
    b[m - 1] = csub(x[m], x[R - m]);
    sum = cadd(sum, a[m - 1]);
  }
  float2 y[R];
  y[0] = sum;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    float2 re = x[0], im = make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const int j = (m * k) % R;
      const float c = kRoots<R>.c[j], sn = kRoots<R>.s[j];
      re = make_float2(fmaf(a[m - 1].x, c, re.x), fmaf(a[m - 1].y, c, re.y));
      im = make_float2(fmaf(b[m - 1].x, sn, im.x), fmaf(b[m - 1].y, sn, im.y));
    }
    const float2 t = mul_mi<INV>(im);     // -i im (forward) or +i im (inverse)
    y[k] = cadd(re, t);
    y[R - k] = csub(re, t);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = y[k];
}

template <> TACAW_HD void dft<3, false>(float2* x) { dft_prime<3, false>(x); }
template <> TACAW_HD void dft<3, true>(float2* x) { dft_prime<3, true>(x); }
template <> TACAW_HD void dft<5, false>(float2* x) { dft_prime<5, false>(x); }
template <> TACAW_HD void dft<5, true>(float2* x) { dft_prime<5, true>(x); }
template <> TACAW_HD void dft<7, false>(float2* x) { dft_prime<7, false>(x); }
template <> TACAW_HD void dft<7, true>(float2* x) { dft_prime<7, true>(x); }

// modular inverse of a mod m (gcd 1) at compile time
constexpr int ct_inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

// N = R1 R2 with gcd(R1, R2) = 1 (Good and Thomas): n = (R2 n1 + R1 n2) mod N and k the number
// with k = k1 mod R1, k = k2 mod R2; then X_k = sum_n1 W_R1^(n1 k1) sum_n2 W_R2^(n2 k2) x_n, with
// no twiddle factors between the two sets of short transforms
template <int R1, int R2, bool INV> TACAW_HD void dft_pfa(float2* x) {
  constexpr int N = R1 * R2;
  constexpr int E1 = R2 * ct_inv_mod(R2 % R1, R1), E2 = R1 * ct_inv_mod(R1 % R2, R2);
  float2 y[N];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    float2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = x[(R2 * n1 + R1 * n2) % N];
    dft<R2, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = t[k2];
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    float2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 * R2 + k2];
    dft<R1, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) x[(k1 * E1 + k2 * E2) % N] = t[k1];
  }
}

// N = R1 R2 (Cooley and Tukey): n = n1 + R1 n2, k = R2 k1 + k2;
// X_k = sum_n1 W_R1^(n1 k1) W_N^(n1 k2) sum_n2 W_R2^(n2 k2) x_n
template <int R1, int R2, bool INV> TACAW_HD void dft_ct(float2* x) {
  constexpr int N = R1 * R2;
  float2 y[N];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    float2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = x[n1 + R1 * n2];
    dft<R2, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = (n1 * k2 == 0) ? t[k2] : cmul(t[k2], root<N, INV>(n1 * k2));
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    float2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 * R2 + k2];
    dft<R1, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) x[R2 * k1 + k2] = t[k1];
  }
}

template <> TACAW_HD void dft<10, false>(float2* x) { dft_pfa<2, 5, false>(x); }
template <> TACAW_HD void dft<10, true>(float2* x) { dft_pfa<2, 5, true>(x); }
template <> TACAW_HD void dft<14, false>(float2* x) { dft_pfa<2, 7, false>(x); }
template <> TACAW_HD void dft<14, true>(float2* x) { dft_pfa<2, 7, true>(x); }
template <> TACAW_HD void dft<20, false>(float2* x) { dft_pfa<4, 5, false>(x); }
template <> TACAW_HD void dft<20, true>(float2* x) { dft_pfa<4, 5, true>(x); }
template <> TACAW_HD void dft<28, false>(float2* x) { dft_pfa<4, 7, false>(x); }
template <> TACAW_HD void dft<28, true>(float2* x) { dft_pfa<4, 7, true>(x); }
template <> TACAW_HD void dft<25, false>(float2* x) { dft_ct<5, 5, false>(x); }
template <> TACAW_HD void dft<25, true>(float2* x) { dft_ct<5, 5, true>(x); }
template <> TACAW_HD void dft<35, false>(float2* x) { dft_pfa<5, 7, false>(x); }
template <> TACAW_HD void dft<35, true>(float2* x) { dft_pfa<5, 7, true>(x); }
template <> TACAW_HD void dft<40, false>(float2* x) { dft_pfa<8, 5, false>(x); }
template <> TACAW_HD void dft<40, true>(float2* x) { dft_pfa<8, 5, true>(x); }

// sin(pi x), cos(pi x) for an exactly representable rational x (twiddle generation)
TACAW_HD void sincospi_f(float x, float* s, float* c) {
#if defined(__HIP_DEVICE_COMPILE__)
  *s = sinpif(x);
  *c = cospif(x);
#else
  double a = 3.14159265358979323846 * (double)x;
  *s = (float)__builtin_sin(a);
  *c = (float)__builtin_cos(a);
#endif
}

// sin x and cos x for the transmission phase sigma V_s.  Reduction by k = nearest integer to
// x / (pi/2): for |x| <= 8192 with pi/2 split into three floats (Cody and Waite), each step one
// fused multiply-add; beyond (never reached by physical potentials, kept exact for any input) in
// float64 with pi/2 split into two doubles.  Then Taylor polynomials on |r| <= pi/4 (truncation
// below 2e-9) and the quadrant's sign/swap.  NaN and infinite x give NaN.
TACAW_HD void sincos_phase(float x, float* s, float* c) {
  constexpr double kHalfPi = 1.57079632679489661923;
  constexpr float P1 = (float)kHalfPi;
  constexpr float P2 = (float)(kHalfPi - (double)P1);
  constexpr float P3 = (float)(kHalfPi - (double)P1 - (double)P2);
  float r;
  int q;
  if (fabsf(x) <= 8192.0f) {
    const float k = rintf(x * (float)(1.0 / kHalfPi));
    r = fmaf(-k, P1, x);
    r = fmaf(-k, P2, r);
    r = fmaf(-k, P3, r);
    q = (int)k & 3;
  } else {
    constexpr double D1 = 1.5707963267948966;          // pi/2 rounded to double
    constexpr double D2 = 6.123233995736766e-17;       // pi/2 - D1
    const double xd = (double)x;
    const double kd = rint(xd * (1.0 / kHalfPi));
    r = (float)fma(-kd, D2, fma(-kd, D1, xd));
    q = (int)(kd - 4.0 * floor(kd * 0.25));          // kd mod 4 (exact: kd is an integer)
  }
  const float r2 = r * r;
  const float sp = r + r * r2 * fmaf(r2, fmaf(r2, fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f),
                                               1.0f / 120.0f), -1.0f / 6.0f);
  const float cp = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f),
                                                   -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
  const float ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// exp(-2 pi i m U / 2^32) for signed index m.  The phase m U is exact in 32-bit fixed point (turns);
// its nearest quarter turn q comes from integer rounding, the remainder r (|r| <= pi/4) is converted
// to radians once, and sin r, cos r are Taylor polynomials (truncation below 2e-9; the remainder's
// conversion costs at most 1e-7 rad), placed in the quadrant by swaps and signs.
TACAW_HD float2 phase_factor(int m, unsigned U) {
  const unsigned ph = (unsigned)m * U;
  const unsigned q = (ph + 0x20000000u) >> 30;
  const float r = (float)(int)(ph - (q << 30)) * 1.46291807926715968e-9f;   // 2 pi / 2^32
  const float r2 = r * r;
  const float sp = r + r * r2 * fmaf(r2, fmaf(r2, fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f),
                                               1.0f / 120.0f), -1.0f / 6.0f);
  const float cp = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f),
                                                   -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
  const float ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
  const float s = (q & 2) ? -ss : ss, c = ((q + 1) & 2) ? -cc : cc;
  return make_float2(c, -s);
}

// ---------------------------------------------------------------------------------------------
// Plans

template <int N_, int L_, int... Rs> struct Plan {
  static constexpr int N = N_;
  static constexpr int L = L_;
  static constexpr int E = N_ / L_;
  static constexpr int LINES = 64 / L_;       // whole lines per wavefront
  static constexpr bool FULL = (64 % L_) == 0;   // the lines fill the wavefront
  static constexpr bool POW2 = (N_ & (N_ - 1)) == 0;
  static_assert(L_ >= 1 && L_ <= 64 && (N_ % L_) == 0, "lanes per line must divide N, at most 64");
  static_assert((1 * ... * Rs) == N_, "radices must multiply to N");
  static constexpr int radix(int k) {
    int rs[] = {Rs...};
    return rs[k];
  }
  static constexpr int NR = (int)sizeof...(Rs);
  // the last radix may leave a remainder in E (in-place LDS stage); all others divide E
  static constexpr bool LDS_LAST = (E % radix(NR - 1)) != 0;
  static constexpr bool radices_ok() {
    for (int k = 0; k + 1 < NR; ++k)
      if (E % radix(k) != 0) return false;
    return !LDS_LAST || NR >= 2;
  }
  static_assert(radices_ok(), "every radix but the last must divide E");
  // lengths that are not powers of two take every twiddle from the LDS root table
  static constexpr int TABN = POW2 ? 0 : N_;
  TACAW_HD static int pad(int p) {
    if constexpr (POW2) return p + (p >> 3);
    else return p;
  }
  static_assert(!LDS_LAST || !POW2, "an LDS last stage needs the root table");
  static constexpr int twiddle_count() {
    if (!POW2) return 0;
    int ns = 1, total = 0;
    for (int k = 0; k < NR; ++k) {
      if (ns > 1 && E % radix(k) == 0) total += (E / radix(k)) * (radix(k) - 1);
      ns *= radix(k);
    }
    return total;
  }
  static constexpr int NTW = twiddle_count() > 0 ? twiddle_count() : 1;
  // LDS words (float2) per line: room for the exchange padding p + p/8, rounded up to 1 mod 16
  // so that 16 adjacent lines staged side by side (column tiles) fall in 16 distinct bank pairs
  static constexpr int LDS_LINE = ((N_ + N_ / 8 + 2 + 14) / 16) * 16 + 1;
};

TACAW_HD int lds_pad(int p) { return p + (p >> 3); }

// LDS position of element p of an N-point line: one pad word per 8 for powers of two (their
// strides are multiples of 8, so the padded addresses stay affine in the register index); no
// padding otherwise (lane counts such as 28 or 50 would make every register need its own address)
template <int N> TACAW_HD int pad_of(int p) {
  if constexpr ((N & (N - 1)) == 0) return lds_pad(p);
  else return p;
}

// Twiddles of one lane kept in an LDS table laid out [k][L]: entry k of lane l at k * L + l, so
// the lanes of a line read consecutive words and the lines of a wave share them.
struct TwStrided {
  const float2* p;   // table + l
  int stride;        // L
  TACAW_HD float2 operator[](int k) const { return p[k * stride]; }
};

// butterflies of one stage for one lane l; v holds E values striped, tw[TO + ...] the stage's
// twiddles (a register array or an accessor) for power-of-two lengths, tab the root table otherwise
template <int N, int L, int R, int NS, bool INV, int TO = 0, class TW>
TACAW_HD void stage_compute(float2* v, const TW& tw, const float2* tab = nullptr, int l = 0) {
  constexpr int E = N / L, B = E / R;
  constexpr bool TABLE = (N & (N - 1)) != 0;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    float2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[i + B * r];
    if constexpr (NS > 1) {
      const int m = TABLE ? (l + L * i) % NS : 0;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = TABLE ? tab[m * r * (N / (NS * R))] : tw[TO + i * (R - 1) + r - 1];
        x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
      }
    }
    dft<R, INV>(x);
#pragma unroll
    for (int r = 0; r < R; ++r) v[i + B * r] = x[r];
  }
}

// the same stage transposed: butterflies first, then the twiddles (as a matrix, B T becomes T B;
// the small DFTs are symmetric).  Run in reverse order with inverted exchanges, the stages of a
// plan compute the same transform (the DFT matrix is symmetric).
template <int N, int L, int R, int NS, bool INV, int TO = 0, class TW>
TACAW_HD void stage_compute_T(float2* v, const TW& tw) {
  constexpr int E = N / L, B = E / R;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    float2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[i + B * r];
    dft<R, INV>(x);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[TO + i * (R - 1) + r - 1];
        x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[i + B * r] = x[r];
  }
}

// destination of output r of butterfly i of lane l in a radix-R stage with span NS
template <int N, int L, int R, int NS> TACAW_HD int stage_out_pos(int l, int i, int r) {
  int b = l + L * i;
  return (b / NS) * NS * R + (b % NS) + r * NS;
}

// forward twiddles of one stage for lane l (conjugated on use for the inverse transform)
template <int N, int L, int R, int NS> TACAW_HD void stage_twiddles(float2* tw, int l) {
  constexpr int E = N / L, B = E / R;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    int b = l + L * i;
    int m = b % NS;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      // angle = -2 pi m r / (NS R) -> sinpi/cospi argument -(m r) / (NS R / 2) (exact in float
      // for power-of-two lengths)
      float xarg = ((NS * R) % 2 == 0) ? -(float)(m * r) / (float)(NS * R / 2)
                                       : -2.0f * (float)(m * r) / (float)(NS * R);
      float s, c;
      sincospi_f(xarg, &s, &c);
      tw[i * (R - 1) + r - 1] = make_float2(c, s);
    }
  }
}

template <int N, int L, int NS, int R, int... Rest>
TACAW_HD void plan_twiddles_rec(float2* tw, int l) {
  constexpr int E = N / L;
  if constexpr (NS > 1 && E % R == 0 && (N & (N - 1)) == 0) {
    stage_twiddles<N, L, R, NS>(tw, l);
    tw += (E / R) * (R - 1);
  }
  if constexpr (sizeof...(Rest) > 0) plan_twiddles_rec<N, L, NS * R, Rest...>(tw, l);
}

// In-place last stage of radix R (R need not divide E) for lane l of a line held in lds: the
// N/R butterflies b read and write b + (N/R) r; lane l takes b = l + L i.  tab[m] = exp(-2 pi i
// m / N); b r < N, so no reduction is needed.
template <int N, int L, int R, bool INV>
TACAW_HD void lds_stage_lane(float2* lds, const float2* tab, int l) {
  constexpr int NS = N / R;
  constexpr int ROUNDS = (NS + L - 1) / L;
#pragma unroll
  for (int i = 0; i < ROUNDS; ++i) {
    const int b = l + L * i;
    if ((NS % L) == 0 || i + 1 < ROUNDS || b < NS) {
      float2 x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = lds[pad_of<N>(b + NS * r)];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tab[b * r];
        x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
      }
      dft<R, INV>(x);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[pad_of<N>(b + NS * r)] = x[r];
    }
  }
}

// whether a plan's remaining radices are exactly one radix that leaves a remainder in E
template <int E, int... Rest> constexpr bool next_is_lds_stage() {
  if constexpr (sizeof...(Rest) == 1) return ((E % Rest) + ...) != 0;
  else return false;
}
template <int... Rest> constexpr int only_radix() { return (Rest + ...); }

// Split-layout transforms of a line spread over a workgroup, for three-stage plans with one
// butterfly per lane and stage (E = R1 = R2 = R3, L = R1 R2: 512 = 8 x 8 x 8 on 64 lanes).  Write
// a lane as l = R1 h + d.  In the first exchange lane l reads only positions = d (mod R1); the
// second exchange writes and reads only such positions, and each is read by a lane with the same
// d.  So the first stage may run on a lane numbering lo chosen for the loads (any lane of the
// line), the exchange re-distributes the line to a numbering lx under which one wavefront holds
// every h of its d, and the second exchange then stays inside that wavefront (no barrier).  The
// inverse transform runs the same flow backwards (transposed stages, exchanges inverted), so its
// only workgroup exchange is its last, which hands the line back to the numbering lo for the
// stores.  Steps are per lane; the caller orders them:
//   forward:  fwd1(lo) | barrier | fwd2(lx) | wave order | fwd3(lx)
//   inverse:  inv1(lx) | wave order | inv2(lx) | barrier | inv3(lo)
// fwd1/fwd2/fwd3/inv1/inv2 use region A of the line, inv2/inv3 region B (inv2 writes B only at
// positions of its own d).  Twiddles are the plan's (PlanOps::twiddles) for lane lx.
template <class P> struct SplitFFT {
  static constexpr int N = P::N, L = P::L, E = P::E;
  static constexpr int R1 = P::radix(0), R2 = P::radix(1), R3 = P::NR == 3 ? P::radix(2) : 0;
  static constexpr bool OK = P::POW2 && P::NR == 3 && E == R1 && E == R2 && E == R3 && L == R1 * R2;
  // lane lo: the first stage (no twiddles) and the first exchange's writes
  TACAW_HD static void fwd1(float2* v, float2* A, int lo) {
    stage_compute<N, L, R1, 1, false>(v, (const float2*)nullptr, nullptr, lo);
#pragma unroll
    for (int r = 0; r < R1; ++r) A[pad_of<N>(stage_out_pos<N, L, R1, 1>(lo, 0, r))] = v[r];
  }
  // lane lx: the first exchange's reads, the second stage, the second exchange's writes (into the
  // same region: Ain = Aout in the kernels, where all lanes of a wavefront read before any writes)
  template <class TW>
  TACAW_HD static void fwd2(float2* v, const TW& tw, const float2* Ain, float2* Aout, int lx) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = Ain[pad_of<N>(lx + L * j)];
    stage_compute<N, L, R2, R1, false, 0>(v, tw, nullptr, lx);
#pragma unroll
    for (int r = 0; r < R2; ++r) Aout[pad_of<N>(stage_out_pos<N, L, R2, R1>(lx, 0, r))] = v[r];
  }
  // lane lx: the second exchange's reads and the last stage (output k = lx + L j in v[j])
  template <class TW> TACAW_HD static void fwd3(float2* v, const TW& tw, const float2* A, int lx) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = A[pad_of<N>(lx + L * j)];
    stage_compute<N, L, R3, R1 * R2, false, R2 - 1>(v, tw, nullptr, lx);
  }
  // inverse (unnormalised), input element k = lx + L j in v[j]
  template <class TW> TACAW_HD static void inv1(float2* v, const TW& tw, float2* A, int lx) {
    stage_compute_T<N, L, R3, R1 * R2, true, R2 - 1>(v, tw);
#pragma unroll
    for (int j = 0; j < E; ++j) A[pad_of<N>(lx + L * j)] = v[j];
  }
  template <class TW>
  TACAW_HD static void inv2(float2* v, const TW& tw, const float2* A, float2* B, int lx) {
#pragma unroll
    for (int r = 0; r < R2; ++r) v[r] = A[pad_of<N>(stage_out_pos<N, L, R2, R1>(lx, 0, r))];
    stage_compute_T<N, L, R2, R1, true, 0>(v, tw);
#pragma unroll
    for (int j = 0; j < E; ++j) B[pad_of<N>(lx + L * j)] = v[j];
  }
  // lane lo: output element lo + L j in v[j]
  TACAW_HD static void inv3(float2* v, const float2* B, int lo) {
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = B[pad_of<N>(stage_out_pos<N, L, R1, 1>(lo, 0, r))];
    stage_compute_T<N, L, R1, 1, true>(v, (const float2*)nullptr);
  }
};

template <class P> struct PlanOps;
template <int N, int L, int... Rs> struct PlanOps<Plan<N, L, Rs...>> {
  TACAW_HD static void twiddles(float2* tw, int l) { plan_twiddles_rec<N, L, 1, Rs...>(tw, l); }
};

#if defined(__HIPCC__)
// intra-wave ordering point for LDS exchanges: the lines of a wave never share LDS, and DS
// instructions of one wave execute in order, so only compiler reordering must be prevented
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Band pruning (PRUNE bit 0: the two middle registers E/2-1 and E/2 of the input are zero;
// bit 1: those registers of the output are not wanted and are returned as zero).  With striped
// storage they hold the indices N/2 - L .. N/2 + L - 1, the middle of the axis, which a band limit
// below N/2 - L removes.  The constants let the compiler drop the work on them.
template <int E, int PRUNE> __device__ __forceinline__ void prune_mid(float2* v, int bit) {
  if constexpr (E >= 4) {
    if (PRUNE & bit) {
      v[E / 2 - 1] = make_float2(0.f, 0.f);
      v[E / 2] = make_float2(0.f, 0.f);
    }
  }
}

template <int N, int L, bool INV, int NS, int PRUNE, int TO, class TW, int R, int... Rest>
__device__ __forceinline__ void fft_rec(float2* v, const TW& tw, float2* lds, int l,
                                        const float2* tab) {
  constexpr int E = N / L, B = E / R;
  if constexpr (NS == 1) prune_mid<E, PRUNE>(v, 1);
  stage_compute<N, L, R, NS, INV, TO>(v, tw, tab, l);
  if constexpr (sizeof...(Rest) > 0) {
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[pad_of<N>(stage_out_pos<N, L, R, NS>(l, i, r))] = v[i + B * r];
    wave_lds_sync();
    if constexpr (next_is_lds_stage<E, Rest...>()) {
      lds_stage_lane<N, L, only_radix<Rest...>(), INV>(lds, tab, l);
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = lds[pad_of<N>(l + L * j)];
      prune_mid<E, PRUNE>(v, 2);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = lds[pad_of<N>(l + L * j)];
      fft_rec<N, L, INV, NS * R, PRUNE, (NS > 1) ? TO + B * (R - 1) : TO, TW, Rest...>(v, tw, lds, l,
                                                                                     tab);
    }
  } else {
    prune_mid<E, PRUNE>(v, 2);
  }
}

// Workgroup variant: the L lanes of a line may sit in different wavefronts, so every exchange is a
// workgroup barrier.  Exchanges alternate between two LDS regions (running parity `buf`); a region
// is rewritten only two exchanges after it was read, with a barrier in between, so one barrier per
// exchange suffices.  With lds1 == lds0 (single buffer) a second barrier guards the rewrite.
// (An LDS last stage runs in place between the exchange's write and its read, with a barrier on
// either side; the region's reuse distance is unchanged.)
template <int N, int L, bool INV, int NS, int PRUNE, int TO, class TW, int R, int... Rest>
__device__ __forceinline__ void fft_block_rec(float2* v, const TW& tw, float2* lds0, float2* lds1,
                                              int l, int& buf, const float2* tab) {
  constexpr int E = N / L, B = E / R;
  static_assert(E % R == 0, "register stages take radices that divide E");
  if constexpr (NS == 1) prune_mid<E, PRUNE>(v, 1);
  stage_compute<N, L, R, NS, INV, TO>(v, tw, tab, l);
  if constexpr (sizeof...(Rest) > 0) {
    float2* lds = buf ? lds1 : lds0;
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[pad_of<N>(stage_out_pos<N, L, R, NS>(l, i, r))] = v[i + B * r];
    __syncthreads();
    if constexpr (next_is_lds_stage<E, Rest...>()) {
      lds_stage_lane<N, L, only_radix<Rest...>(), INV>(lds, tab, l);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = lds[pad_of<N>(l + L * j)];
      if (lds0 == lds1) __syncthreads();
      buf ^= 1;
      prune_mid<E, PRUNE>(v, 2);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = lds[pad_of<N>(l + L * j)];
      if (lds0 == lds1) __syncthreads();
      buf ^= 1;
      fft_block_rec<N, L, INV, NS * R, PRUNE, (NS > 1) ? TO + B * (R - 1) : TO, TW, Rest...>(
          v, tw, lds0, lds1, l, buf, tab);
    }
  } else {
    prune_mid<E, PRUNE>(v, 2);
  }
}

// The workgroup's table of N-th roots of unity for a plan with an LDS last stage.  Every thread of
// the workgroup calls fft_table_init once before the first transform (it ends with a barrier).
template <class P> __device__ __forceinline__ float2* fft_table_storage() {
  __shared__ float2 t[P::TABN > 0 ? P::TABN : 1];
  return t;
}
template <class P> __device__ __forceinline__ const float2* fft_table_init() {
  if constexpr (P::TABN > 0) {
    float2* t = fft_table_storage<P>();
    for (int m = (int)threadIdx.x; m < P::N; m += (int)blockDim.x) {
      double sn, cs;
      sincospi(-2.0 * (double)m / (double)P::N, &sn, &cs);
      t[m] = make_float2((float)cs, (float)sn);
    }
    __syncthreads();
    return t;
  } else {
    return nullptr;
  }
}

template <class P> struct FFT;
template <int N, int L, int... Rs> struct FFT<Plan<N, L, Rs...>> {
  // unnormalised transform of one line held striped in v; lds = this line's exchange region;
  // tab = the workgroup's root table (plans with an LDS last stage only)
  template <bool INV, int PRUNE = 0, class TW>
  __device__ __forceinline__ static void run(float2* v, const TW& tw, float2* lds, int l,
                                             const float2* tab = nullptr) {
    fft_rec<N, L, INV, 1, PRUNE, 0, TW, Rs...>(v, tw, lds, l, tab);
  }
  // same transform when the line's lanes span several wavefronts of the workgroup
  template <bool INV, int PRUNE = 0, class TW>
  __device__ __forceinline__ static void run_block(float2* v, const TW& tw, float2* lds0,
                                                   float2* lds1, int l, int& buf,
                                                   const float2* tab = nullptr) {
    fft_block_rec<N, L, INV, 1, PRUNE, 0, TW, Rs...>(v, tw, lds0, lds1, l, buf, tab);
  }
};
#endif

}  // namespace tacaw
