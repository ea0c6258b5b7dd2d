// Reads cases "D reach c0..c3 m[a][0..3]... p[a][0..3]... outside par" (hex words)
// from stdin and prints the code words and packed counts of codes16<D>.
#include <cstdio>
#include <cstdint>
#include "group_codes.h"

template <int D>
static void run(const uint32_t* c, const uint32_t (*m)[4], const uint32_t (*p)[4], uint32_t outside, uint64_t par,
                int reach) {
  uint32_t out[4];
  const uint64_t cnt = gcodes::codes16<D>(c, m, p, outside, par, reach, out);
  std::printf("%08x %08x %08x %08x %016llx\n", out[0], out[1], out[2], out[3], (unsigned long long)cnt);
}

int main() {
  int D, reach;
  while (std::scanf("%d %d", &D, &reach) == 2) {
    uint32_t c[4], m[3][4] = {}, p[3][4] = {};
    unsigned long long par;
    unsigned outside;
    int ok = 1;
    for (int q = 0; q < 4; q++) ok &= std::scanf("%x", &c[q]) == 1;
    for (int a = 0; a < D; a++)
      for (int q = 0; q < 4; q++) ok &= std::scanf("%x", &m[a][q]) == 1;
    for (int a = 0; a < D; a++)
      for (int q = 0; q < 4; q++) ok &= std::scanf("%x", &p[a][q]) == 1;
    ok &= std::scanf("%x", &outside) == 1;
    ok &= std::scanf("%llx", &par) == 1;
    if (!ok) return 1;
    if (D == 1) run<1>(c, m, p, outside, par, reach);
    else if (D == 2) run<2>(c, m, p, outside, par, reach);
    else run<3>(c, m, p, outside, par, reach);
  }
  return 0;
}
