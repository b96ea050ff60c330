// Host-only parts of the library, with no HIP dependency: scenario-tree
// validation (section 4.1, Fig. 1), checks of the problem data, the offline
// factorisation of Alg. 1 in FP64, ||L|| from the block-diagonal structure of
// L (remark after its definition in section 5.2), the exact nested AV@R cost
// of a trajectory (section 4.2, eq. original-problem) and the work-item list
// of the dataflow sweeps. Built into libspock.so and, on its own, into a CPU
// driver run under AddressSanitizer and UndefinedBehaviorSanitizer.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/spock.h"

namespace spk {

struct Tree {
  int nn = 0, nl = 0, N = 0;
  std::vector<int> anc, fc, nch, stage;
  std::vector<int> stage_off;  // [N+2]: nodes of stage t are [stage_off[t], stage_off[t+1])
  std::vector<double> prob, pcond;
};

// Builds and validates a tree from breadth-first ancestors and node
// probabilities. Returns SPOCK_OK, SPOCK_EINVAL, SPOCK_ETREE or SPOCK_EPROB.
int build_tree(int32_t nn, const int32_t* anc, const double* prob, Tree& T);

// Finite data, positive weights, ordered boxes, a in [0, 1]. Returns SPOCK_OK,
// SPOCK_EINVAL or SPOCK_EBOX (dimensions are checked by the caller).
int check_problem_data(const Tree& T, const spock_problem_data& d);

// Alg. 1 in FP64, stage N-1 down to 0 (nodes of a stage in parallel): per
// nonleaf node the inverse of R~ and K, per child Abar = A + B K, per node P,
// and per nonleaf node W = sum_c Abar^c' P^c B^c. Row-major per node:
// Abar [nn][nx][nx], K [nl][nu][nx], Rinv [nl][nu][nu], W [nl][nx][nu],
// P [nn][nx][nx]. Returns SPOCK_OK or SPOCK_EFACTOR.
struct Factor {
  std::vector<double> P, Abar, K, Rinv, W;
};
int factor_alg1(const Tree& T, const spock_problem_data& d, Factor& F);

// ||L|| as the largest spectral norm of its blocks (closed forms per block).
double norm_L_blocks(const Tree& T, const spock_problem_data& d);

// Exact nested AV@R cost of (x, u) ([nn][nx], [nl][nu] row-major): leaves
// x'Q_N x; each nonleaf node the AV@R of its children's stage cost plus cost
// to go, with conditional probabilities.
double nested_cost(const Tree& T, int nx, int nu, const double* q, const double* r, const double* qN,
                   const double* a_risk, const std::vector<double>& x, const std::vector<double>& u);

// Work items of the dataflow sweeps with nc children per chunk: backward
// items (families in reverse breadth-first order, chunks in increasing
// order), then forward items (breadth-first); item code = family * chunk_codes
// + chunk. pbase[i] is the first partial-sum slot of a family with several
// chunks; nslots the number of slots. Returns SPOCK_OK, or SPOCK_EINVAL when a
// family needs chunk_codes chunks or more.
int build_flow_items(const Tree& T, int nc, int chunk_codes, std::vector<int>& items, std::vector<int>& pbase,
                     int& nslots, int& nbwd);

// Parallel loop over [0, n) on up to 16 host threads.
template <typename F>
void parallel_for(int n, F&& f) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hw ? hw : 1, 16u);
  if (n < 64 || nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  nt = std::min(nt, n);
  std::vector<std::thread> th;
  for (int w = 0; w < nt; ++w)
    th.emplace_back([&, w]() {
      for (int i = w; i < n; i += nt) f(i);
    });
  for (auto& t : th) t.join();
}

}  // namespace spk
