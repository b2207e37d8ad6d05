// Host-side placement of reactions on lanes and of species in the per-cell LDS arrays.
//
// The reaction lanes of a segment read the concentrations of the four species of their
// reaction and add their rate into those species' accumulators: one LDS instruction per
// species slot serves L reactions at once (reaction j = lane + L i in iteration i).  Two
// lanes of one instruction that touch different addresses in the same LDS bank, or that
// add into the same accumulator, are serialised.  Neither the order in which reactions
// are assigned to (iteration, lane) positions nor the position of a species in the LDS
// arrays changes what is computed (only the order of the production sums), so both are
// chosen here to spread every instruction's addresses over the banks.
//
// Cost model: the LDS serves an instruction in passes of G lanes over B four-byte banks;
// a pass costs the largest number of distinct addresses that fall in one bank, and an
// accumulate pass at least the largest number of lanes adding into one address.  With two
// accumulator copies (the mixed layout) lanes of even and odd index accumulate into
// different copies, so their addresses differ for the same species.  The
// search minimises the sum over the two geometries (B, G) = (32, 16) and (64, 32) by
// simulated annealing over swaps of two reaction positions or two species positions,
// with a fixed seed (the placement is a deterministic function of the mechanism).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace rok4e {

struct Placement {
  std::vector<int> order;   // position p (p < nr) -> reaction index
  std::vector<int> pos;     // species k (k <= ns, ns = absent slot) -> LDS position
};

class PlacementSearch {
 public:
  // slots: [nr][4] species of reactant 0, 1, product 0, 1 (ns for an absent slot);
  // L: lanes per segment; word: bytes of one concentration entry (8 or 4); copy_dw:
  // distance in four-byte words between the two accumulator copies (0: one copy).
  PlacementSearch(int ns, int nr, const std::vector<int>& slots, int L, int word, int copy_dw)
      : ns_(ns), nr_(nr), L_(L), word_(word), copy_dw_(copy_dw), slots_(slots) {
    order_.resize(nr);
    for (int j = 0; j < nr; ++j) order_[j] = j;
    pos_.resize(ns + 1);
    for (int k = 0; k <= ns; ++k) pos_[k] = k;
    stamp_.assign(2 * (ns + 1), 0);
    mult_.assign(2 * (ns + 1), 0);
    rstamp_.assign(ns + 1, 0);
    n_it_ = (nr + L - 1) / L;
    for (int g = 0; g < 2; ++g) {
      const int G = std::min(kGeom[g].G, L);
      groups_[g] = L / G;
    }
    cost_.assign((size_t)n_it_ * 8, 0);
    total_ = 0;
    for (int it = 0; it < n_it_; ++it) {
      cost_[it] = iter_cost(it);
      total_ += cost_[it];
    }
  }

  long total() const { return total_; }

  Placement run(long steps, uint64_t seed) {
    uint64_t s = seed;
    auto next = [&s]() {   // splitmix64
      uint64_t z = (s += 0x9E3779B97F4A7C15ull);
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      return z ^ (z >> 31);
    };
    auto unif = [&next]() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); };
    std::vector<int> best_order = order_, best_pos = pos_;
    long best = total_;
    const double T0 = 2.0, T1 = 0.05;
    for (long step = 0; step < steps && nr_ > 1; ++step) {
      const double temp = T0 * std::pow(T1 / T0, (double)step / (double)steps);
      if (unif() < 0.75) {
        const int a = (int)(next() % (uint64_t)nr_), b = (int)(next() % (uint64_t)nr_);
        const int ia = a / L_, ib = b / L_;
        if (ia == ib) continue;   // same instruction: the cost does not change
        std::swap(order_[a], order_[b]);
        const long ca = iter_cost(ia), cb = iter_cost(ib);
        const long d = ca + cb - cost_[ia] - cost_[ib];
        if (d <= 0 || unif() < std::exp(-(double)d / temp)) {
          cost_[ia] = ca;
          cost_[ib] = cb;
          total_ += d;
        } else {
          std::swap(order_[a], order_[b]);
        }
      } else {
        if (ns_ < 2) continue;
        const int a = (int)(next() % (uint64_t)ns_), b = (int)(next() % (uint64_t)ns_);
        if (a == b) continue;
        std::swap(pos_[a], pos_[b]);
        long t = 0;
        std::vector<long> nc(n_it_);
        for (int it = 0; it < n_it_; ++it) {
          nc[it] = iter_cost(it);
          t += nc[it];
        }
        const long d = t - total_;
        if (d <= 0 || unif() < std::exp(-(double)d / temp)) {
          for (int it = 0; it < n_it_; ++it) cost_[it] = nc[it];
          total_ = t;
        } else {
          std::swap(pos_[a], pos_[b]);
        }
      }
      if (total_ < best) {
        best = total_;
        best_order = order_;
        best_pos = pos_;
      }
    }
    order_ = best_order;
    pos_ = best_pos;
    total_ = best;
    return Placement{order_, pos_};
  }

 private:
  struct Geom {
    int B, G;
  };
  static constexpr Geom kGeom[2] = {{32, 16}, {64, 32}};

  // Cost of iteration it (positions it L .. it L + L - 1) over the four slots, both
  // geometries, reads and accumulates.
  long iter_cost(int it) const {
    long c = 0;
    const int words = word_ / 4;
    for (int gi = 0; gi < 2; ++gi) {
      const int B = kGeom[gi].B, G = std::min(kGeom[gi].G, L_);
      for (int g = 0; g < groups_[gi]; ++g) {
        for (int sl = 0; sl < 4; ++sl) {
          ++gen_;
          int rmax = 0, amax = 0, bmax = 0;
          int rload[64] = {0}, aload[64] = {0};
          for (int l = g * G; l < (g + 1) * G; ++l) {
            const int p = it * L_ + l;
            if (p >= nr_) break;
            const int a = pos_[slots_[order_[p] * 4 + sl]];
            if (rstamp_[a] != gen_) {   // first lane reading this concentration
              rstamp_[a] = gen_;
              rmax = std::max(rmax, ++rload[(a * words) % B]);
            }
            const int c = copy_dw_ ? (l & 1) : 0;   // accumulator copy of this lane
            const int ka = a + c * (ns_ + 1);
            if (stamp_[ka] != gen_) {   // first lane adding into this address
              stamp_[ka] = gen_;
              mult_[ka] = 1;
              bmax = std::max(bmax, ++aload[(a * 2 + c * copy_dw_) % B]);
            } else {
              ++mult_[ka];
            }
            amax = std::max(amax, mult_[ka]);
          }
          c += rmax + std::max(amax, bmax);
        }
      }
    }
    return c;
  }

  int ns_, nr_, L_, word_, copy_dw_, n_it_;
  int groups_[2];
  std::vector<int> slots_, order_, pos_;
  mutable std::vector<int> stamp_, mult_, rstamp_;
  mutable int gen_ = 0;
  std::vector<long> cost_;
  long total_;
};

}  // namespace rok4e
