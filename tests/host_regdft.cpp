// Host build of the register DFTs of csrc/cx.hpp (compiled with the
// stand-in header of tests/host_shim): for every supported length N and both
// directions, prints N, DIR and the DFT of a fixed input, one value a line,
// for tests/test_host_regdft.py to compare with numpy's FFT.
#include <cmath>
#include <cstdio>

#include "../paper_1501_06286_amd/csrc/cx.hpp"

using namespace qmc;

template <int N, int DIR>
void emit() {
  cx<double> v[N];
  for (int i = 0; i < N; ++i) v[i] = {std::sin(1.3 * i + 0.2), std::cos(0.7 * i * i + 1.0)};
  reg_fft<double, N, DIR>(v);
  std::printf("N %d %d\n", N, DIR);
  for (int i = 0; i < N; ++i) std::printf("%.17g %.17g\n", v[i].x, v[i].y);
}
template <int N>
void both() {
  emit<N, -1>();
  emit<N, +1>();
}

int main() {
  both<1>(); both<2>(); both<4>(); both<8>(); both<16>(); both<32>(); both<64>();
  both<3>(); both<6>(); both<12>(); both<24>(); both<48>(); both<96>();
  both<5>(); both<10>(); both<20>(); both<40>(); both<80>();
  return 0;
}
