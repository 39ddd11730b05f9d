// CPU emulation of the wave-level Stockham FFT in fft.hpp.
//
// Every lane of a line is emulated in turn with the very same per-lane functions the kernels use
// (stage_compute, stage_out_pos, stage_twiddles, pad_of); the LDS exchange is an array.  The
// result of each plan, forward and inverse, is compared with a double-precision DFT.  Prints one
// line per plan and exits non-zero on any mismatch.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "fft.hpp"
#include "plans.hpp"

using namespace tacaw;

template <int N, int L, bool INV, int NS, int R, int... Rest>
static void emu_rec(std::vector<float2>& v, std::vector<std::vector<float2>>& tw, int twoff,
                    std::vector<float2>& lds, const std::vector<float2>& tab) {
  constexpr int E = N / L, B = E / R;
  for (int l = 0; l < L; ++l) {
    const float2* t = &tw[l][twoff];
    stage_compute<N, L, R, NS, INV>(&v[l * E], t, tab.data(), l);
  }
  if constexpr (sizeof...(Rest) > 0) {
    for (int l = 0; l < L; ++l)
      for (int i = 0; i < B; ++i)
        for (int r = 0; r < R; ++r)
          lds[pad_of<N>(stage_out_pos<N, L, R, NS>(l, i, r))] = v[l * E + i + B * r];
    if constexpr (next_is_lds_stage<E, Rest...>()) {
      // in-place last stage: the lanes' butterflies touch disjoint positions
      for (int l = 0; l < L; ++l) lds_stage_lane<N, L, only_radix<Rest...>(), INV>(lds.data(), tab.data(), l);
      for (int l = 0; l < L; ++l)
        for (int j = 0; j < E; ++j) v[l * E + j] = lds[pad_of<N>(l + L * j)];
    } else {
      for (int l = 0; l < L; ++l)
        for (int j = 0; j < E; ++j) v[l * E + j] = lds[pad_of<N>(l + L * j)];
      emu_rec<N, L, INV, NS * R, Rest...>(v, tw, (NS > 1) ? twoff + B * (R - 1) : twoff, lds, tab);
    }
  }
}

// every LDS position a lane stage touches lies inside the line's region
template <int N, int L, int R> static bool lds_stage_in_bounds(int lds_line) {
  constexpr int NS = N / R, ROUNDS = (NS + L - 1) / L;
  for (int l = 0; l < L; ++l)
    for (int i = 0; i < ROUNDS; ++i) {
      const int b = l + L * i;
      if (!((NS % L) == 0 || i + 1 < ROUNDS || b < NS)) continue;
      if (b >= NS) return false;
      for (int r = 0; r < R; ++r)
        if (pad_of<N>(b + NS * r) >= lds_line || b * r >= N) return false;
    }
  return true;
}

template <class P> struct Emu;
template <int N, int L, int... Rs> struct Emu<Plan<N, L, Rs...>> {
  template <bool INV> static double run(unsigned seed) {
    using PL = Plan<N, L, Rs...>;
    constexpr int E = N / L;
    std::mt19937 g(seed);
    std::normal_distribution<float> d;
    std::vector<std::complex<double>> x(N);
    for (auto& z : x) z = {d(g), d(g)};
    std::vector<float2> v(L * E);
    for (int l = 0; l < L; ++l)
      for (int j = 0; j < E; ++j) {
        auto z = x[l + L * j];
        v[l * E + j] = make_float2((float)z.real(), (float)z.imag());
      }
    std::vector<std::vector<float2>> tw(L, std::vector<float2>(PL::NTW));
    for (int l = 0; l < L; ++l) PlanOps<PL>::twiddles(tw[l].data(), l);
    std::vector<float2> lds(PL::LDS_LINE);
    std::vector<float2> tab(N);
    for (int m = 0; m < N; ++m)
      tab[m] = make_float2((float)std::cos(-2.0 * M_PI * m / N), (float)std::sin(-2.0 * M_PI * m / N));
    if constexpr (PL::LDS_LAST) {
      if (!lds_stage_in_bounds<N, L, PL::radix(PL::NR - 1)>(PL::LDS_LINE)) return 1e30;
    }
    emu_rec<N, L, INV, 1, Rs...>(v, tw, 0, lds, tab);
    double err = 0, nrm = 0;
    const double sgn = INV ? 1.0 : -1.0;
    for (int k = 0; k < N; ++k) {
      std::complex<double> acc = 0;
      for (int n = 0; n < N; ++n) {
        long long kn = (long long)k * n % N;
        acc += x[n] * std::polar(1.0, sgn * 2.0 * M_PI * (double)kn / N);
      }
      float2 got = v[(k % L) * E + k / L];
      err += std::norm(std::complex<double>(got.x, got.y) - acc);
      nrm += std::norm(acc);
    }
    return std::sqrt(err / nrm);
  }
};

template <class P> static int check(const char* name) {
  double ef = Emu<P>::template run<false>(7), ei = Emu<P>::template run<true>(11);
  bool ok = ef < 2e-6 && ei < 2e-6;
  std::printf("%-28s N=%5d L=%3d  fwd rel-L2 %.2e  inv rel-L2 %.2e  %s\n", name, P::N, P::L, ef, ei,
              ok ? "ok" : "FAIL");
  // the exchange writes of every stage stay inside the line's region too
  if (P::pad(P::N - 1) >= P::LDS_LINE) {
    std::printf("%-28s LDS line too short\n", name);
    return 1;
  }
  return ok ? 0 : 1;
}

// The split-layout transforms: every lane step in the order the kernels run them (lanes lo and lx
// each range over the whole line), checked against a double-precision DFT both ways, and the
// residue property that makes the second exchange wave-local: every position lane lx touches in
// the steps between the workgroup exchanges is congruent to lx modulo R1.
template <class P> static int check_split(const char* name) {
  using S = SplitFFT<P>;
  constexpr int N = P::N, L = P::L, E = P::E;
  static_assert(S::OK, "not a split plan");
  bool resid = true;
  for (int lx = 0; lx < L; ++lx)
    for (int j = 0; j < E; ++j) {
      resid &= (lx + L * j) % S::R1 == lx % S::R1;
      resid &= stage_out_pos<N, L, S::R2, S::R1>(lx, 0, j) % S::R1 == lx % S::R1;
    }
  std::mt19937 g(23);
  std::normal_distribution<float> d;
  double worst = 0;
  for (int dir = 0; dir < 2; ++dir) {
    std::vector<std::complex<double>> x(N);
    for (auto& z : x) z = {d(g), d(g)};
    std::vector<float2> v(L * E), A(P::LDS_LINE), B(P::LDS_LINE);
    std::vector<std::vector<float2>> tw(L, std::vector<float2>(P::NTW));
    for (int l = 0; l < L; ++l) PlanOps<P>::twiddles(tw[l].data(), l);
    for (int l = 0; l < L; ++l)
      for (int j = 0; j < E; ++j) v[l * E + j] = make_float2((float)x[l + L * j].real(), (float)x[l + L * j].imag());
    if (dir == 0) {
      for (int l = 0; l < L; ++l) S::fwd1(&v[l * E], A.data(), l);
      const std::vector<float2> A1 = A;   // every lane reads before any lane writes
      for (int l = 0; l < L; ++l) S::fwd2(&v[l * E], tw[l].data(), A1.data(), A.data(), l);
      for (int l = 0; l < L; ++l) S::fwd3(&v[l * E], tw[l].data(), A.data(), l);
    } else {
      for (int l = 0; l < L; ++l) S::inv1(&v[l * E], tw[l].data(), A.data(), l);
      for (int l = 0; l < L; ++l) S::inv2(&v[l * E], tw[l].data(), A.data(), B.data(), l);
      for (int l = 0; l < L; ++l) S::inv3(&v[l * E], B.data(), l);
    }
    const double sgn = dir == 1 ? 1.0 : -1.0;
    double err = 0, nrm = 0;
    for (int k = 0; k < N; ++k) {
      std::complex<double> acc = 0;
      for (int n = 0; n < N; ++n)
        acc += x[n] * std::polar(1.0, sgn * 2.0 * M_PI * (double)((long long)k * n % N) / N);
      const float2 got = v[(k % L) * E + k / L];
      err += std::norm(std::complex<double>(got.x, got.y) - acc);
      nrm += std::norm(acc);
    }
    worst = std::max(worst, std::sqrt(err / nrm));
  }
  const bool ok = resid && worst < 2e-6;
  std::printf("%-28s N=%5d L=%3d  split fwd/inv rel-L2 %.2e  residues %s  %s\n", name, N, L, worst,
              resid ? "ok" : "BAD", ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}

// sincos_phase against double precision: moderate arguments, quadrant boundaries, the fallback
static int check_sincos() {
  double worst = 0;
  auto probe = [&](float x) {
    float s, c;
    sincos_phase(x, &s, &c);
    worst = std::max(worst, std::max(std::fabs(s - std::sin((double)x)),
                                     std::fabs(c - std::cos((double)x))));
  };
  for (int i = -2000000; i <= 2000000; ++i) probe((float)i * 1.5e-4f);          // [-300, 300]
  for (int k = -4000; k <= 4000; ++k)
    for (int d = -3; d <= 3; ++d) probe(std::nextafter((float)(k * M_PI_4), d > 0 ? 1e9f : -1e9f) + d * 1e-6f);
  for (int i = 0; i < 1000; ++i) probe(8000.0f + (float)i * 1.37f);             // both branches
  for (int i = 0; i < 1400; ++i) probe((i & 1 ? -1.0f : 1.0f) * 1.0e4f * std::pow(1.013f, (float)i));  // to ~7e11
  const bool ok = worst < 1e-6;
  std::printf("%-28s max abs error %.2e  %s\n", "sincos_phase", worst, ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}

// phase_factor against exp(-2 pi i (m U mod 2^32) / 2^32) in double: random fixed-point coordinates
// and signed indices up to +-512, plus the phases nearest every quadrant and octant boundary
static int check_phase_factor() {
  double worst = 0;
  auto probe = [&](int m, unsigned U) {
    const float2 f = phase_factor(m, U);
    const unsigned ph = (unsigned)m * U;
    const double a = -2.0 * M_PI * (double)ph / 4294967296.0;
    worst = std::max(worst, std::max(std::fabs(f.x - std::cos(a)), std::fabs(f.y - std::sin(a))));
  };
  std::mt19937 g(11);
  for (int i = 0; i < 2000000; ++i) probe((int)(g() % 1024u) - 512, (unsigned)g());
  for (unsigned b = 0; b < 8; ++b)
    for (int d = -40; d <= 40; ++d) probe(1, b * 0x20000000u + (unsigned)d);
  const bool ok = worst < 2.5e-7;
  std::printf("%-28s max abs error %.2e  %s\n", "phase_factor", worst, ok ? "ok" : "FAIL");
  return ok ? 0 : 1;
}

int main() {
  int bad = check_sincos() + check_phase_factor();
#define TACAW_CHECK_PLAN(NAME, ...) bad += check<__VA_ARGS__>(NAME);
  TACAW_FOR_EACH_PLAN(TACAW_CHECK_PLAN)
  bad += check_split<P512a>("n512 L64 8x8x8 split");
  std::printf("%s\n", bad ? "FFT host check FAILED" : "FFT host check passed");
  return bad ? 1 : 0;
}
