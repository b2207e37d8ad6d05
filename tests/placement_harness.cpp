// Test harness for the host-side LDS placement search (no GPU): reads "ns nr" and the
// [nr][4] slot table from stdin, runs the search with the given lanes, word size,
// accumulator-copy distance, steps and seed, and prints the initial and final model
// cost, the reaction order and the species positions.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rok4e_placement.hpp"

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  const int L = std::atoi(argv[1]), word = std::atoi(argv[2]), copy_dw = std::atoi(argv[3]);
  const long steps = std::atol(argv[4]);
  const unsigned long long seed = std::strtoull(argv[5], nullptr, 0);
  int ns = 0, nr = 0;
  if (std::scanf("%d %d", &ns, &nr) != 2) return 3;
  std::vector<int> slots(4 * (size_t)nr);
  for (int& x : slots)
    if (std::scanf("%d", &x) != 1) return 3;
  rok4e::PlacementSearch search(ns, nr, slots, L, word, copy_dw);
  const long c0 = search.total();
  const rok4e::Placement p = search.run(steps, seed);
  std::printf("%ld %ld\n", c0, search.total());
  for (int x : p.order) std::printf("%d ", x);
  std::printf("\n");
  for (int x : p.pos) std::printf("%d ", x);
  std::printf("\n");
  return 0;
}
