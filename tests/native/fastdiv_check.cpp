// Host check of FastDiv (internal.h): floor(n / d) by multiply-high and shift
// equals integer division for every divisor tried (all of 2..4096, the
// lattice extents of every order up to 2^20 elements per direction, powers
// of two and their neighbours) at the numerators where an error would show
// first: multiples of d and their neighbours, the top of the 31-bit range,
// and a seeded random sample.
#include <cstdio>
#include <random>
#include <vector>

#include "internal.h"

int main() {
  std::vector<int> ds;
  for (int d = 2; d <= 4096; ++d) ds.push_back(d);
  for (int p = 1; p <= 8; ++p)
    for (int n = 1; n <= (1 << 20); n = n * 3 / 2 + 1) ds.push_back(n * p + 1);
  for (int k = 2; k < 31; ++k)
    for (int o = -1; o <= 1; ++o) ds.push_back((1 << k) + o);
  ds.push_back(0x7fffffff);
  std::mt19937_64 g(15940);
  long long bad = 0, checked = 0;
  for (int d : ds) {
    if (d < 2) continue;
    const pafem::FastDiv f(d);
    auto chk = [&](long long n) {
      if (n < 0 || n > 0x7fffffffLL) return;
      ++checked;
      if (f.div((int)n) != (int)(n / d)) ++bad;
    };
    for (long long k = 0; k <= 2000; ++k)
      for (int o = -1; o <= 1; ++o) chk(k * d + o);
    for (long long k = (0x7fffffffLL / d) - 2000; k <= 0x7fffffffLL / d + 1; ++k)
      for (int o = -1; o <= 1; ++o) chk(k * d + o);
    for (int t = 0; t < 2000; ++t) chk((long long)(g() & 0x7fffffff));
    chk(0x7fffffff);
  }
  std::printf("divisors=%zu checked=%lld bad=%lld\n", ds.size(), checked, bad);
  return bad == 0 ? 0 : 1;
}
