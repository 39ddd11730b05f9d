// The FFT plans compiled into the library: (line length N, lanes per line L, radices).
// Several plans exist per N; the autotuner picks among them at run time.  Plan index 0 of each N
// is the default when no tuning result is available.
#pragma once
#include "fft.hpp"

namespace tacaw {
using P16a = Plan<16, 2, 8, 2>;
using P16b = Plan<16, 4, 4, 4>;
using P32a = Plan<32, 4, 8, 4>;
using P32b = Plan<32, 2, 16, 2>;
using P64a = Plan<64, 8, 8, 8>;
using P64b = Plan<64, 4, 16, 4>;
using P128a = Plan<128, 16, 8, 4, 4>;
using P128b = Plan<128, 8, 16, 8>;
using P256a = Plan<256, 32, 8, 8, 4>;
using P256b = Plan<256, 16, 16, 16>;
using P256c = Plan<256, 64, 4, 4, 4, 4>;
using P512a = Plan<512, 64, 8, 8, 8>;
using P512b = Plan<512, 32, 16, 8, 4>;
using P1024a = Plan<1024, 64, 16, 16, 4>;
using P1024b = Plan<1024, 64, 16, 4, 16>;
// lengths with odd factors: register stages whose radices divide E (their product may exceed E),
// then an in-place LDS stage of the remaining radix
using P560a = Plan<560, 28, 4, 5, 4, 7>;     // E = 20, 2 lines per wavefront (lanes 56..63 idle)
using P560b = Plan<560, 56, 2, 5, 2, 2, 14>; // E = 10, 1 line per wavefront (lanes 56..63 idle)
using P560c = Plan<560, 28, 20, 4, 7>;       // E = 20: one exchange fewer than P560a
using P560d = Plan<560, 28, 20, 28>;         // E = 20: one exchange, then an LDS radix-28 stage
using P1000a = Plan<1000, 50, 4, 5, 5, 10>;  // E = 20, 1 line per wavefront (lanes 50..63 idle)
using P1000b = Plan<1000, 50, 10, 10, 10>;   // E = 20, register stages only
}  // namespace tacaw

// X(name, plan) for every plan
#define TACAW_FOR_EACH_PLAN(X)                                                                     \
  X("n16 L2 8x2", tacaw::P16a) X("n16 L4 4x4", tacaw::P16b) X("n32 L4 8x4", tacaw::P32a)        \
  X("n32 L2 16x2", tacaw::P32b) X("n64 L8 8x8", tacaw::P64a) X("n64 L4 16x4", tacaw::P64b)       \
  X("n128 L16 8x4x4", tacaw::P128a) X("n128 L8 16x8", tacaw::P128b)                              \
  X("n256 L32 8x8x4", tacaw::P256a) X("n256 L16 16x16", tacaw::P256b)                            \
  X("n256 L64 4x4x4x4", tacaw::P256c) X("n512 L64 8x8x8", tacaw::P512a)                          \
  X("n512 L32 16x8x4", tacaw::P512b) X("n1024 L64 16x16x4", tacaw::P1024a)                       \
  X("n1024 L64 16x4x16", tacaw::P1024b) X("n560 L28 4x5x4x7", tacaw::P560a)                        \
  X("n560 L56 2x5x2x2x14", tacaw::P560b) X("n560 L28 20x4x7", tacaw::P560c)                     \
  X("n560 L28 20x28", tacaw::P560d)                                                              \
  X("n1000 L50 4x5x5x10", tacaw::P1000a) X("n1000 L50 10x10x10", tacaw::P1000b)
