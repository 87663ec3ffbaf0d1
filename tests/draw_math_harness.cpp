// Host harness for tpmc_math.hpp: for every k read from stdin (one decimal per
// line) prints log_draw(k), then sin and cos of 2 pi (k + 1/2) 2^-32 from
// sincos_2pi_draw with a table of the 256 angles built here in long double.
#include <cmath>
#include <cstdio>

#include "tpmc_math.hpp"

int main() {
  static double tab[512];
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < 256; ++j) {
    tab[2 * j] = (double)sinl(2.0L * pi * j / 256.0L);
    tab[2 * j + 1] = (double)cosl(2.0L * pi * j / 256.0L);
  }
  unsigned long long k;
  while (std::scanf("%llu", &k) == 1) {
    double s, c;
    tpmc::sincos_2pi_draw(tab, (uint32_t)k, s, c);
    std::printf("%a %a %a\n", tpmc::log_draw((uint32_t)k), s, c);
  }
  return 0;
}
