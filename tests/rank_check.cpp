// Host build of the eigenvalue ranking used by the small-SVD finishing kernel:
// reads "l v0 v1 ..." lines (values as text; "nan", "inf", "-inf" allowed) and
// prints the ranks of each line, one line per input line.
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../paper_1907_06470_amd/csrc/rank.h"

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream is(line);
    int l = 0;
    is >> l;
    std::vector<double> v(l);
    for (int i = 0; i < l; ++i) {
      std::string t;
      is >> t;
      v[i] = std::strtod(t.c_str(), nullptr);
    }
    std::vector<double> lv(l);
    for (int i = 0; i < l; ++i) lv[i] = rsvd::nan_as_low(v[i]);
    for (int i = 0; i < l; ++i) std::printf(i ? " %d" : "%d", rsvd::desc_rank(lv.data(), l, i));
    std::printf("\n");
  }
  return 0;
}
