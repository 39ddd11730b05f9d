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

// sin x and cos x for the transmission phase sigma V_s (moderate |x|).  Reduction by k = nearest
// integer to x / (pi/2) with pi/2 split into three floats (Cody and Waite), each step one fused
// multiply-add, then Taylor polynomials on |r| <= pi/4 (truncation below 2e-9) and the quadrant's
// sign/swap.  Beyond |x| = 8192 the library routine is used.
TACAW_HD void sincos_phase(float x, float* s, float* c) {
  constexpr double kHalfPi = 1.57079632679489661923;
  constexpr float P1 = (float)kHalfPi;
  constexpr float P2 = (float)(kHalfPi - (double)P1);
  constexpr float P3 = (float)(kHalfPi - (double)P1 - (double)P2);
  if (!(fabsf(x) <= 8192.0f)) {
#if defined(__HIP_DEVICE_COMPILE__)
    sincosf(x, s, c);
#else
    *s = (float)__builtin_sin((double)x);
    *c = (float)__builtin_cos((double)x);
#endif
    return;
  }
  const float k = rintf(x * (float)(1.0 / kHalfPi));
  float r = fmaf(-k, P1, x);
  r = fmaf(-k, P2, r);
  r = fmaf(-k, P3, r);
  const float r2 = r * r;
  const float sp = r + r * r2 * fmaf(r2, fmaf(r2, fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f),
                                               1.0f / 120.0f), -1.0f / 6.0f);
  const float cp = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f),
                                                   -1.0f / 720.0f), 1.0f / 24.0f), -0.5f), 1.0f);
  const int q = (int)k & 3;
  const float ss = (q & 1) ? cp : sp, cc = (q & 1) ? sp : cp;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// ---------------------------------------------------------------------------------------------
// Plans

template <int N_, int L_, int... Rs> struct Plan {
  static constexpr int N = N_;
  static constexpr int L = L_;
  static constexpr int E = N_ / L_;
  static constexpr int LINES = 64 / L_;       // lines per wavefront
  static_assert(L_ >= 1 && L_ <= 64 && (64 % L_) == 0, "lanes per line must divide 64");
  static_assert((1 * ... * Rs) == N_, "radices must multiply to N");
  static_assert((((E % Rs) == 0) && ...), "every radix must divide E");
  static constexpr int twiddle_count() {
    int ns = 1, total = 0;
    int rs[] = {Rs...};
    for (int k = 0; k < (int)sizeof...(Rs); ++k) {
      if (ns > 1) total += (E / rs[k]) * (rs[k] - 1);
      ns *= rs[k];
    }
    return total;
  }
  static constexpr int NTW = twiddle_count() > 0 ? twiddle_count() : 1;
  // LDS words (float2) per line: room for the exchange padding p + p/8, rounded up to 1 mod 16
  // so that 16 adjacent lines staged side by side (column tiles) fall in 16 distinct bank pairs
  static constexpr int LDS_LINE = ((N_ + N_ / 8 + 2 + 14) / 16) * 16 + 1;
};

TACAW_HD int lds_pad(int p) { return p + (p >> 3); }

// butterflies of one stage for one lane; v holds E values striped, tw the stage's twiddles
template <int N, int L, int R, int NS, bool INV>
TACAW_HD void stage_compute(float2* v, const float2* tw) {
  constexpr int E = N / L, B = E / R;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    float2 x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[i + B * r];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r)
        x[r] = INV ? cmulc(x[r], tw[i * (R - 1) + r - 1]) : cmul(x[r], tw[i * (R - 1) + r - 1]);
    }
    dft<R, INV>(x);
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
      // angle = -2 pi m r / (NS R) -> sinpi/cospi argument -(m r) / (NS R / 2), exact in float
      float xarg = -(float)(m * r) / (float)(NS * R / 2);
      float s, c;
      sincospi_f(xarg, &s, &c);
      tw[i * (R - 1) + r - 1] = make_float2(c, s);
    }
  }
}

template <int N, int L, int NS, int R, int... Rest>
TACAW_HD void plan_twiddles_rec(float2* tw, int l) {
  constexpr int E = N / L;
  if constexpr (NS > 1) {
    stage_twiddles<N, L, R, NS>(tw, l);
    tw += (E / R) * (R - 1);
  }
  if constexpr (sizeof...(Rest) > 0) plan_twiddles_rec<N, L, NS * R, Rest...>(tw, l);
}

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

template <int N, int L, bool INV, int NS, int PRUNE, int R, int... Rest>
__device__ __forceinline__ void fft_rec(float2* v, const float2* tw, float2* lds, int l) {
  constexpr int E = N / L, B = E / R;
  if constexpr (NS == 1) prune_mid<E, PRUNE>(v, 1);
  stage_compute<N, L, R, NS, INV>(v, tw);
  if constexpr (sizeof...(Rest) > 0) {
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(stage_out_pos<N, L, R, NS>(l, i, r))] = v[i + B * r];
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = lds[lds_pad(l + L * j)];
    fft_rec<N, L, INV, NS * R, PRUNE, Rest...>(v, (NS > 1) ? tw + B * (R - 1) : tw, lds, l);
  } else {
    prune_mid<E, PRUNE>(v, 2);
  }
}

// Workgroup variant: the L lanes of a line may sit in different wavefronts, so every exchange is a
// workgroup barrier.  Exchanges alternate between two LDS regions (running parity `buf`); a region
// is rewritten only two exchanges after it was read, with a barrier in between, so one barrier per
// exchange suffices.  With lds1 == lds0 (single buffer) a second barrier guards the rewrite.
template <int N, int L, bool INV, int NS, int PRUNE, int R, int... Rest>
__device__ __forceinline__ void fft_block_rec(float2* v, const float2* tw, float2* lds0,
                                              float2* lds1, int l, int& buf) {
  constexpr int E = N / L, B = E / R;
  if constexpr (NS == 1) prune_mid<E, PRUNE>(v, 1);
  stage_compute<N, L, R, NS, INV>(v, tw);
  if constexpr (sizeof...(Rest) > 0) {
    float2* lds = buf ? lds1 : lds0;
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(stage_out_pos<N, L, R, NS>(l, i, r))] = v[i + B * r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = lds[lds_pad(l + L * j)];
    if (lds0 == lds1) __syncthreads();
    buf ^= 1;
    fft_block_rec<N, L, INV, NS * R, PRUNE, Rest...>(v, (NS > 1) ? tw + B * (R - 1) : tw, lds0, lds1,
                                                     l, buf);
  } else {
    prune_mid<E, PRUNE>(v, 2);
  }
}

template <class P> struct FFT;
template <int N, int L, int... Rs> struct FFT<Plan<N, L, Rs...>> {
  // unnormalised transform of one line held striped in v; lds = this line's exchange region
  template <bool INV, int PRUNE = 0>
  __device__ __forceinline__ static void run(float2* v, const float2* tw, float2* lds, int l) {
    fft_rec<N, L, INV, 1, PRUNE, Rs...>(v, tw, lds, l);
  }
  // same transform when the line's lanes span several wavefronts of the workgroup
  template <bool INV, int PRUNE = 0>
  __device__ __forceinline__ static void run_block(float2* v, const float2* tw, float2* lds0,
                                                   float2* lds1, int l, int& buf) {
    fft_block_rec<N, L, INV, 1, PRUNE, Rs...>(v, tw, lds0, lds1, l, buf);
  }
};
#endif

}  // namespace tacaw
