// Prints the LDS layout of the swizzled FFT lengths (dh_fft.hpp): for each
// length, whether it is swizzled, the transform stride, the plan's radices,
// then the slot of every element. Host-only build; used by test_lds_layout.py.
#include "dh_fft.hpp"
#include <cstdio>

template <int N>
void dump() {
  using P = dh::FftPlan<N>;
  std::printf("N %d SWZ %d STRIDE %d R %d %d %d\n", N, (int)dh::Lds<N>::SWZ, dh::Lds<N>::STRIDE, P::R0, P::R1, P::R2);
  for (int i = 0; i < N; ++i) std::printf("%d%c", dh::swz<N>(i), i + 1 < N ? ' ' : '\n');
}

int main() {
  dump<512>();
  dump<1024>();
  dump<2048>();
  return 0;
}
