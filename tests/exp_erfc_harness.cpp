// Host harness for exp_erfc_grid (tpmc_math.hpp): builds the table of
// exp(-y_j^2) and erfc(y_j) at y_j = j / 256 in long double, then for every y
// read from stdin (hexadecimal float, one per line) prints exp(-y^2) and
// erfc(y) with 8, 9, 10 and 11 series terms (the library uses 10), then y
// rounded to FP32 and erfcx32 there.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "tpmc_math.hpp"

int main() {
  static double tab[2 * tpmc::kExpErfcN];
  for (int j = 0; j < tpmc::kExpErfcN; ++j) {
    const long double y = (long double)j / 256.0L;
    tab[2 * j] = (double)expl(-y * y);
    tab[2 * j + 1] = (double)erfcl(y);
  }
  char buf[128];
  while (std::scanf("%127s", buf) == 1) {
    const double y = std::strtod(buf, nullptr);
    double e8, t8, e9, t9, e10, t10, e11, t11;
    tpmc::exp_erfc_grid<8>(tab, y, e8, t8);
    tpmc::exp_erfc_grid<9>(tab, y, e9, t9);
    tpmc::exp_erfc_grid<10>(tab, y, e10, t10);
    tpmc::exp_erfc_grid<11>(tab, y, e11, t11);
    const float yf = (float)y;
    std::printf("%a %a %a %a %a %a %a %a %a %a\n", e8, t8, e9, t9, e10, t10, e11, t11, (double)yf,
                (double)tpmc::erfcx32(yf));
  }
  return 0;
}
