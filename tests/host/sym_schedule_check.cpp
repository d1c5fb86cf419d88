// Checks the push order of the split 32^3 kernel's pair-symmetric form, built against
// the library's own table builder (split32_sym_tables). For each configuration it
// prints one line: nwg nk nb shift pairs pushes faults. Faults counted:
//   - an ordered (target, source) pair not covered exactly once, either directly (the
//     target runs the source) or through a push (the source, as a target, runs the target
//     as its source and pushes the conjugate term);
//   - a push where the table has none, or none where it has one;
//   - a mirror copy whose ranks are not 0 .. n - 1 once each, or whose order is not the
//     key order (round, pair within the target, CU pair within the XCD), the order that
//     keeps the kernel's waits free of deadlock;
//   - a count table that disagrees with the pushes.
// The schedule restated here is the kernel's: CU pair slot = t mod (nwg/2) runs targets
// t = slot + round (nwg/2) on XCD slot / (nwg/16); target (k, i) at pair s = d nb + m
// runs source ((k + d) mod nk, ((i >> shift) + m) mod nb), d = 0 .. nk/2, and pushes for
// 1 <= d <= (nk - 1)/2.
#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

namespace fockmi {
void split32_sym_tables(int nwg, int nk, int nb, int shift, std::vector<int>* rank, std::vector<int>* cnt);
}

static long check(int nwg, int nk, int nb, int shift) {
  std::vector<int> rank, cnt;
  fockmi::split32_sym_tables(nwg, nk, nb, shift, &rank, &cnt);
  const int npairs = nwg / 2, per_x = npairs / 8, nt = nk * nb, ndelta = nk / 2 + 1, npush = (nk - 1) / 2;
  const int ns = ndelta * nb;
  long faults = 0, pushes = 0;
  if ((long)rank.size() != (long)nt * ns || (long)cnt.size() != 8L * nt) return 1;
  std::vector<int> cover((size_t)nt * nt, 0);
  std::map<std::pair<long, int>, std::tuple<int, int, int>> key_of;  // (copy, rank) -> key
  for (int t = 0; t < nt; ++t) {
    const int slot = t % npairs, round = t / npairs, x = slot / per_x, pp = slot % per_x;
    const int k = t / nb, i = t % nb;
    for (int s = 0; s < ns; ++s) {
      const int d = s / nb, m = s % nb;
      const int src = ((k + d) % nk) * nb + ((i >> shift) + m) % nb;
      cover[(size_t)t * nt + src] += 1;
      const bool push = d >= 1 && d <= npush;
      const int r = rank[(size_t)t * ns + s];
      if (push != (r >= 0)) ++faults;
      if (!push || r < 0) continue;
      ++pushes;
      cover[(size_t)src * nt + t] += 1;
      const long copy = (long)x * nt + src;
      if (!key_of.emplace(std::make_pair(copy, r), std::make_tuple(round, s, pp)).second) ++faults;
    }
  }
  for (int v : cover) faults += v != 1;
  long total = 0;
  for (int x = 0; x < 8; ++x)
    for (int b = 0; b < nt; ++b) {
      const long copy = (long)x * nt + b;
      const int n = cnt[copy];
      total += n;
      for (int r = 0; r < n; ++r) {
        auto it = key_of.find({copy, r});
        if (it == key_of.end()) {
          ++faults;
          continue;
        }
        if (r > 0) {
          auto prev = key_of.find({copy, r - 1});
          if (prev != key_of.end() && !(prev->second < it->second)) ++faults;
        }
      }
    }
  if (total != pushes || (long)key_of.size() != pushes) ++faults;
  std::printf("%d %d %d %d %ld %ld %ld\n", nwg, nk, nb, shift, (long)nt * ns, pushes, faults);
  return faults;
}

int main() {
  const int cfg[][3] = {{256, 216, 16}, {256, 8, 4}, {256, 8, 3}, {256, 27, 10}, {256, 3, 1},
                        {256, 4, 3}, {32, 9, 5}, {256, 125, 16}, {64, 6, 20}};
  long faults = 0;
  for (const auto& c : cfg)
    for (int shift : {0, 1, 2, 5}) faults += check(c[0], c[1], c[2], shift);
  return faults != 0;
}
