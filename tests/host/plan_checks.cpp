// Host-side checks of the plan builder, compiled with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_plan_host_sanitizers.py: plans for
// dense (4-bit codes) and sparse (variable-list) rankings, every precision,
// and the size errors; every doubled basis monomial must rank inside [0, M),
// and the gram's tile list must hold each upper-triangle tile exactly once.
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "sos_internal.h"

// plan.cpp's only outside dependencies (the error channel of api.cpp, and the
// destructor that releases timing events, none of which these plans hold)
namespace sos {
int set_error(int code, const std::string& msg) { (void)msg; return code; }
int hip_error(hipError_t e, const char* what) { (void)e; (void)what; return SOS_EHIP; }
}  // namespace sos
sos_plan_s::~sos_plan_s() {}

int main() {
  int bad = 0, bad_tiles = 0, made = 0, refused = 0;
  const int shapes[][2] = {{1, 1}, {2, 1}, {3, 2}, {4, 3}, {6, 4}, {8, 4}, {10, 5}, {12, 3}, {16, 2},
                           {16, 3}, {17, 1}, {17, 2}, {30, 2}, {99, 2}, {40, 3}, {20, 4}, {3, 7},
                           {5, 7}, {2, 8}, {17, 5}, {256, 1}};
  for (const auto& sh : shapes) {
    for (int prec = 0; prec < 3; ++prec) {
      sos_plan_s* p = nullptr;
      if (sos::plan_create(sh[0], sh[1], 23, prec, &p) != 0) {
        ++refused;
        continue;
      }
      ++made;
      std::vector<uint8_t> twice(p->n);
      for (int64_t i = 0; i < p->N; ++i) {
        for (int v = 0; v < p->n; ++v) twice[v] = (uint8_t)(2 * p->basis[i * p->n + v]);
        const int64_t r = sos::rank_closed_form(p->n, 2 * p->d, twice.data());
        if (r < 0 || r >= p->M) ++bad;
      }
      const int T = (int)(p->Np / 256);
      std::vector<int> seen((size_t)T * T, 0);
      if (p->tile_list.size() != (size_t)T * (T + 1) || p->ntiles256 != T * (T + 1) / 2) ++bad_tiles;
      for (size_t t = 0; t + 1 < p->tile_list.size(); t += 2) {
        const int I = p->tile_list[t], J = p->tile_list[t + 1];
        if (I < 0 || I > J || J >= T || seen[(size_t)I * T + J]++) ++bad_tiles;
      }
      delete p;
    }
  }
  std::printf("plans %d refused %d bad ranks %d bad tiles %d\n", made, refused, bad, bad_tiles);
  return bad != 0 || bad_tiles != 0 || made == 0 || refused == 0;
}
