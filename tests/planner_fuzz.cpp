// Sanitizer build of the host planner (built and run by tests/test_planner_fuzz.py
// on the CPU): random layer lists -- valid and invalid -- through validation,
// plan building, the plan description and the flop accounting, so that
// AddressSanitizer and UndefinedBehaviorSanitizer see every path the C ABI's
// circuit creation drives with caller-controlled input.
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "planner.h"

using namespace tqs;

int main(int argc, char **argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 2000;
  std::mt19937_64 rng(20261203);
  auto uni = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
  int built = 0, rejected = 0;
  for (int it = 0; it < iters; ++it) {
    const bool wild = uni(0, 9) == 0;   // one case in ten may hold anything
    const int n = wild ? uni(-2, 33) : uni(1, 20);
    const int nl = uni(0, 24);
    std::vector<LayerSpec> L(nl);
    for (auto &l : L) {
      l.gate = wild ? uni(-3, 20) : uni(0, 16);
      const bool one = l.gate <= 9 || l.gate == 16;
      if (wild) {
        l.pattern = uni(-2, 8);
      } else if (one) {
        l.pattern = uni(0, 3) ? 0 : 1;   // ALL or WIRE
      } else {
        l.pattern = uni(1, 5);
        if ((l.pattern == 4 || l.pattern == 5) && n % 2) l.pattern = 2;
      }
      l.source = wild ? uni(-1, 4) : uni(0, 2);
      l.wire = wild ? uni(-5, 40) : uni(0, std::max(0, n - 1));
      l.wire2 = wild ? uni(-5, 40) : (n > 1 ? (l.wire + uni(1, n - 1)) % n : 0);
      l.offset = wild ? (uni(0, 3) == 0 ? INT32_MAX - uni(0, 64) : uni(-10, 1000)) : uni(0, 200);
      l.fixed = std::uniform_real_distribution<double>(-7, 7)(rng);
      l.fixed2 = uni(0, 2) ? 0.0 : std::uniform_real_distribution<double>(-1, 1)(rng);
      l.fixed3 = uni(0, 2) ? 0.0 : std::uniform_real_distribution<double>(-1, 1)(rng);
    }
    PlanOptions o;
    o.mode = uni(0, 3);
    const int kt[4] = {0, 10, 11, 12};
    o.tile_bits = kt[uni(0, 3)];
    o.hrz = uni(0, 1);
    o.fhwt = uni(0, 1);
    o.diag = uni(0, 1);
    Plan P;
    const std::string e = build_plan(P, n, L.data(), nl, uni(0, 1), o);
    if (!e.empty()) {
      ++rejected;
      continue;
    }
    ++built;
    const std::string d = describe_plan(P);
    double f = 0, b = 0;
    for (size_t p = 0; p < P.passes.size(); ++p) pass_flops(P, (int)p, &f, &b);
    if (d.empty() || f < 0 || b < 0) {
      std::printf("bad plan description\n");
      return 1;
    }
  }
  std::printf("planner fuzz: %d built, %d rejected\n", built, rejected);
  return built > 0 && rejected > 0 ? 0 : 2;
}
