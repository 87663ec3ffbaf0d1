// Host harness for tpmc_math.hpp: prints log_draw(k) in hex for every k read
// from stdin (one decimal per line).
#include <cstdio>

#include "tpmc_math.hpp"

int main() {
  unsigned long long k;
  while (std::scanf("%llu", &k) == 1) std::printf("%a\n", tpmc::log_draw((uint32_t)k));
  return 0;
}
